// Host runtime of the ICNNM library: contexts, HBM budget, tile planning, the
// phase-driven group executor shared by solve / solve_batch / serving, the
// eigenvector learning pre-step and the C ABI of include/icnnm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <list>
#include <set>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/icnnm.h"
#include "admission.h"
#include "icnnm_dev.h"

namespace icnnm {

void sym_eig(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V);

struct Error : std::runtime_error {
  icnnm_status code;
  Error(icnnm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCK(expr)                                                                                  \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess)                                                                            \
      throw Error(ICNNM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));               \
  } while (0)

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------------------ memory budget
struct Budget {
  size_t limit = 0;
  std::atomic<size_t> used{0};
  // When set, allocations are carved from [arena, arena + limit) by bumping `used`
  // (256-byte aligned) and releases are no-ops: no device allocation is made.
  char* arena = nullptr;
  void* alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    if (arena) {
      const size_t off = (used.load() + 255) & ~(size_t)255;
      if (off + bytes > limit)
        throw Error(ICNNM_E_BUDGET, "solver state exceeds the allocation-free scratch maximum of " +
                                        std::to_string(limit >> 20) + " MiB");
      used = off + bytes;
      return arena + off;
    }
    size_t cur = used.load();
    do {
      if (cur + bytes > limit) throw Error(ICNNM_E_BUDGET, "HBM budget exhausted");
    } while (!used.compare_exchange_weak(cur, cur + bytes));
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      used -= bytes;
      (void)hipGetLastError();
      throw Error(ICNNM_E_NOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
    }
    return p;
  }
  void release(void* p, size_t bytes) {
    if (!p || arena) return;
    (void)hipFree(p);
    used -= bytes;
  }
};

struct DevBuf {
  Budget* b = nullptr;
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(); }
  void reset() {
    if (p && b) b->release(p, n);
    p = nullptr;
    n = 0;
  }
  void ensure(Budget* bud, size_t bytes) {
    if (bytes <= n && p) return;
    reset();
    b = bud;
    p = bud->alloc(bytes);
    n = bytes;
  }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

// ------------------------------------------------------------------------------ planning
struct Plan {
  int m[3], k[3], b[3], E[3], nt[3], C[3], goff[3];
  int ntiles, bm, E123, nlblk, nslice;
  int gshift;  // gather-table entries pack (tile index << gshift) | box position
  bool split = false;  // split contractions (64-wide groups, offsets shared by the wavefronts)
  int64_t mtot;
  std::vector<int32_t> gtab;
  size_t state_floats() const;
};

constexpr int kTilesPerSlice = 16;

static int pow2ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// partial sums of the split contractions: 12 slots of one 32x32 accumulator piece
constexpr int kSplitRedFloats = 12 * 16 * 64;

static int lds_forward_floats(const Plan& p, int kp, bool split = false, bool x3 = false) {
  // FP32: halo + offset table; reduced precision: 4-wide expanded halo of 16-bit values
  // (2 floats per position; three such halos in the split-BF16 refresh) + a quarter-size
  // offset table; the larger of the two; then the column and residual partials (and
  // the split form's partial sums)
  const int CG = split ? kColUnit : std::min(kp, kGroup);
  const int nrc = p.bm / kRowUnit, ncc = CG / kColUnit;
  const int h32 = ((p.E123 + 3) & ~3) + kp, hlp = (x3 ? 6 : 2) * p.E123 + kp / 4;
  if (split) return std::max(h32, hlp) + 2 * (2 * nrc) * CG + 4 * nrc * ncc + kSplitRedFloats;
  return std::max(h32, hlp) + 2 * nrc * CG + nrc * ncc;
}

// the line-owning col2im gather: innermost kernel extent 4, innermost tile extent 8,
// at most two box lines per thread
static bool lines_gather_fits(const Plan& p) {
  return p.k[2] == 4 && p.b[2] == 8 && p.E[0] * p.E[1] <= 2 * kThreads;
}

static int lds_adjoint_floats(const Plan& p, int kp, bool split = false) {
  // staged H^T of one round: (offsets per round) x (tile rows + 4); the split form
  // stages 64 offsets in one round, after its partial sums
  if (split) return kColUnit * (p.bm + 4) + kSplitRedFloats;
  const int SGW = std::min(kp, kGroup);
  const int units = (p.bm / kRowUnit) * (SGW / kColUnit);
  const int rounds = units >= 4 ? units / 4 : 1;
  return (SGW / rounds) * (p.bm + 4);
}

// Every admissible tile box with its cost-model estimate, cheapest first (the plans
// are not yet finished: see finish_plan).
static std::vector<std::pair<double, Plan>> plan_candidates(const int m[3], const int k[3], int kp) {
  std::vector<std::pair<double, Plan>> out;
  const int nsg = (kp + kGroup - 1) / kGroup;
  // ICNNM_TILE=b0,b1,b2 forces one tile box (used to compare tile shapes)
  int force[3] = {0, 0, 0};
  if (const char* e = getenv("ICNNM_TILE")) sscanf(e, "%d,%d,%d", &force[0], &force[1], &force[2]);
  for (int bm : {64, 128, 256, 512}) {
    if (kp >= 512 && bm != 128) continue;  // the tiled large-kernel adjoint uses 128-row tiles
    for (int b2 = 1; b2 <= bm; b2 <<= 1) {
      if (b2 > pow2ceil(m[2]) && b2 * pow2ceil(m[1]) * pow2ceil(m[0]) > bm) continue;
      for (int b1 = 1; b1 * b2 <= bm && b1 <= pow2ceil(m[1]); b1 <<= 1) {
        const int b0 = bm / (b1 * b2);
        if (b0 * b1 * b2 != bm || b0 > pow2ceil(m[0])) continue;
        if (force[0] > 0 && (b0 != force[0] || b1 != force[1] || b2 != force[2])) continue;
        Plan p{};
        for (int d = 0; d < 3; ++d) {
          p.m[d] = m[d];
          p.k[d] = k[d];
        }
        p.b[0] = b0;
        p.b[1] = b1;
        p.b[2] = b2;
        p.bm = bm;
        int64_t ntiles = 1;
        for (int d = 0; d < 3; ++d) {
          p.E[d] = p.b[d] + k[d] - 1;
          p.nt[d] = (m[d] + p.b[d] - 1) / p.b[d];
          ntiles *= p.nt[d];
        }
        p.E123 = p.E[0] * p.E[1] * p.E[2];
        p.ntiles = (int)ntiles;
        if (lds_forward_floats(p, kp) * 4 > 150 * 1024) continue;
        {
          // box positions per thread of the col2im gather: 16 (per-unit adjoint),
          // 24 (large-kernel adjoint)
          if (bm / kRowUnit > 4 || p.E123 > (kp >= 512 ? 6144 : 4096)) continue;
          if (lds_adjoint_floats(p, kp) * 4 > 80 * 1024) continue;
        }
        if (p.E[0] > 65535 || p.E[1] > 65535 || p.E[2] > 65535 || ntiles > 65535 * 16) continue;
        // gather-table entries pack (tile index << gshift) | box position into a
        // non-negative int32: gshift bits hold every box position, the rest the tiles
        p.gshift = 1;
        while ((1 << p.gshift) < std::max(p.E[0], std::max(p.E[1], p.E[2]))) ++p.gshift;
        if (std::max(p.nt[0], std::max(p.nt[1], p.nt[2])) > (1 << (31 - p.gshift)) - 1) continue;
        // cost model: rounds of resident workgroups (two per CU, limited by the
        // adjoint's registers) x (units per wavefront + prologue/epilogue overhead),
        // slowed when fewer than two wavefronts per SIMD are resident, times the
        // padding of ragged tiles, the halo traffic and a preference for long
        // innermost tile rows
        const double mt = (double)m[0] * m[1] * m[2];
        const double padded = (double)ntiles * bm / mt;
        const double halo = (double)p.E123 * nsg / (2.0 * bm * kp);
        const double wgs = (double)ntiles * nsg;
        const double slots = 256.0 * 2.0;
        const double rounds = std::ceil(wgs / slots);
        const double upw = (double)(bm / kRowUnit) * (std::min(kp, kGroup) / kColUnit) / 4.0;
        const double eff = wgs >= slots ? 1.0 : 0.5 + 0.5 * wgs / slots;
        const double inner = 1.0 + 0.005 * std::log2(32.0 / std::min(b2, 32));
        // tiles that admit the line-owning col2im gather (innermost kernel extent 4)
        const double gather = (k[2] == 4 && !lines_gather_fits(p)) ? 1.3 : 1.0;
        // 128-row tiles admit the operand-reusing tiled adjoint when kp is a multiple of 256
        const double tiled = (kp % kGroup == 0 && bm != 128) ? 1.3 : 1.0;
        const double cost = rounds * (std::max(upw, 1.0) + 0.5) / eff * padded * (1.0 + halo) * inner * gather * tiled;
        out.emplace_back(cost, p);
      }
    }
  }
  std::stable_sort(out.begin(), out.end(),
                   [](const std::pair<double, Plan>& a, const std::pair<double, Plan>& b) { return a.first < b.first; });
  return out;
}

// sizes and gather tables of a chosen tile box
static void finish_plan(Plan& p, int kp) {
  const int* m = p.m;
  const int* k = p.k;
  p.mtot = (int64_t)m[0] * m[1] * m[2];
  p.nlblk = (int)((p.mtot + kLStepElems - 1) / kLStepElems);
  p.nslice = kp / 4;  // column-norm blocks: kp / 64 column blocks x kColRanges tile ranges
  // gather tables: for each coordinate t of dimension d, the (tile, box position) pairs
  // whose box position (n b - (k - 1) + p) mod m equals t
  int off = 0;
  for (int d = 0; d < 3; ++d) {
    std::vector<std::vector<int32_t>> lists(m[d]);
    for (int n = 0; n < p.nt[d]; ++n)
      for (int q = 0; q < p.E[d]; ++q) {
        int t = n * p.b[d] - (k[d] - 1) + q;
        t %= m[d];
        if (t < 0) t += m[d];
        lists[t].push_back((n << p.gshift) | q);
      }
    int C = 0;
    for (auto& l : lists) C = std::max<int>(C, (int)l.size());
    p.C[d] = C;
    p.goff[d] = off;
    for (auto& l : lists) {
      for (int c = 0; c < C; ++c) p.gtab.push_back(c < (int)l.size() ? l[c] : -1);
    }
    off += m[d] * C;
  }
}

// the cost model's choice
static Plan make_plan(const int m[3], const int k[3], int kp) {
  auto c = plan_candidates(m, k, kp);
  if (c.empty()) throw Error(ICNNM_E_INVALID, "no tile shape fits this problem");
  Plan p = c.front().second;
  finish_plan(p, kp);
  return p;
}

// A member of a joint launch (batch or server group): the kernel variants are chosen
// per launch, so one member with tiles unfit for the tiled adjoint (128 rows) or the
// line gather moves every member to the slower variant; and the launch has the
// workgroups of all members, so a small member gains nothing from smaller tiles.
// Hence the cheapest box that keeps both, when there is one.
static bool keeps_shared_variants(const Plan& p, int kp) {
  return (kp % kGroup != 0 || p.bm == 128) && (p.k[2] != 4 || lines_gather_fits(p));
}

static Plan make_plan_shared(const int m[3], const int k[3], int kp) {
  auto c = plan_candidates(m, k, kp);
  if (c.empty()) throw Error(ICNNM_E_INVALID, "no tile shape fits this problem");
  Plan p = c.front().second;
  for (auto& cp : c)
    if (keeps_shared_variants(cp.second, kp)) {
      p = cp.second;
      break;
    }
  finish_plan(p, kp);
  return p;
}

// the admissible plan with tile box b, or the cost model's choice if b is not admissible
static Plan plan_with_box(const int m[3], const int k[3], int kp, const int b[3]) {
  for (auto& cp : plan_candidates(m, k, kp))
    if (cp.second.b[0] == b[0] && cp.second.b[1] == b[1] && cp.second.b[2] == b[2]) {
      Plan p = cp.second;
      finish_plan(p, kp);
      return p;
    }
  return make_plan(m, k, kp);
}

// Split contractions for an instance solved alone whose launches would otherwise have
// fewer workgroups than the chip has compute units: 64-row tiles, kp a multiple of 128
// (FP32) or 256 (BF16/FP16: their forward contracts 64 offsets per step). ICNNM_SPLIT=0
// or 1 forces the choice where the plan admits the split form.
constexpr int kSplitBelowWorkgroups = 256;

static void decide_split(Plan& p, int kp, int prec) {
  const int nsg = (kp + kGroup - 1) / kGroup;
  bool fits = p.bm == kRowUnit && kp % (prec == kFP32 ? 128 : 256) == 0 &&
              lds_forward_floats(p, kp, true) * 4 <= 150 * 1024 && lds_adjoint_floats(p, kp, true) * 4 <= 150 * 1024;
  bool want = (int64_t)p.ntiles * nsg < kSplitBelowWorkgroups;
  if (const char* e = getenv("ICNNM_SPLIT")) want = atoi(e) != 0;
  p.split = fits && want;
}

// ------------------------------------------------------------------------------ group executor
// One solve state: the device arrays of one instance.
struct Member {
  Plan plan;
  icnnm_params params;
  const float* M = nullptr;
  const uint8_t* mask = nullptr;
  float* Lout = nullptr;
  DevBuf buf;     // all per-instance state, carved below
  InstDev dev{};  // host copy of the descriptor
  int slot = -1;  // index into the group's InstState array
  // serving bookkeeping
  uint64_t ticket = 0;
  double t_submit = 0, t_start = 0;
  int round = 0;  // rounds the member has been part of (its round r runs iteration r)
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// padded kernel size: a multiple of the 64-column wave unit, and of the 256-column
// workgroup group once k exceeds one group
static int padded_k(int k) { return k <= kGroup ? (k + 63) / 64 * 64 : (k + kGroup - 1) / kGroup * kGroup; }

// column groups of the forward and offset groups of the adjoint (halo partials per
// tile): 256 wide, or 64 wide in the split form
static int plan_groups(const Plan& p, int kp) { return p.split ? kp / kColUnit : (kp + kGroup - 1) / kGroup; }

static size_t member_bytes(const Plan& p, int kp, int prec) {
  const int nsg = plan_groups(p, kp), ncg = nsg;
  size_t b = 0;
  const size_t st = (size_t)p.ntiles * p.bm * kp;
  b += align256(st * 4) + align256(st * (prec != kFP32 ? 2 : 4));  // W; U (16 bits in the reduced precisions)
  b += align256((size_t)p.ntiles * nsg * p.E123 * 4);        // part
  b += 2 * align256((size_t)p.ntiles * kp * 4);              // qpart, wpart
  b += align256((size_t)p.ntiles * ncg * 4);                 // rpart
  b += align256((size_t)p.nlblk * 16);                       // dlpart
  b += align256((size_t)(2 * kColRanges * kp + 3 * p.nslice) * 8);  // column sums + scalar partials
  b += align256((size_t)kp * 4);                             // s
  b += align256(p.gtab.size() * 4);                          // gather tables
  if (prec != kFP32) b += 2 * align256((size_t)p.mtot * 4);  // Lprev, T
  return b;
}

// Kernel dimensions the contractions run with. The reduced-precision forward reads
// runs of four consecutive innermost kernel offsets, so for BF16/FP16 the innermost
// kernel extent is padded to a multiple of 4 with offsets whose rows of V are zero:
// A_k'(L) V' = A_k(L) V and A_k'^*(X V'^T) = A_k^*(X V^T) exactly, and the L-step
// keeps dividing by the true k. FP32 runs the kernel as given.
static void contraction_dims(const int kd[3], int prec, int kdp[3]) {
  for (int d = 0; d < 3; ++d) kdp[d] = kd[d];
  if (prec != kFP32) kdp[2] = (kd[2] + 3) / 4 * 4;
}

struct Group {
  Budget* budget;
  int kd[3];   // contraction kernel dimensions (innermost padded for BF16/FP16)
  int kdt[3];  // the kernel's own dimensions
  int k, kt;   // offsets of the contraction kernel; of the kernel itself (the 1/k of the L-step)
  int kp, nsg, ncg, prec;
  const float* Vsrc = nullptr;
  DevBuf Vf, Va, Vp, Vlo_f, Vlo_a, Vlo_p;
  DevBuf Vx_f, Vx_p;  // split-BF16 V (heads, then tails) for the refresh rounds
  DevBuf Vpad;  // V with the zero rows and columns of padded kernel offsets
  bool big = false;  // adjoint tiled for operand reuse: kp a multiple of 256, 128-row tiles
  // refresh rounds of the reduced precisions contracted in split BF16 (the tiled adjoint
  // and the 64-row-unit forward) instead of FP32; ICNNM_REFRESH=fp32 keeps FP32
  bool rx3 = false;
  int lds_fwd_x3 = 0;
  bool split = false;  // split contractions: every member's plan has the split form
  std::vector<Member*> members;
  int capacity;
  DevBuf states;  // InstState[capacity]
  std::vector<int> free_slots;
  DevBuf inst, tiles, lblocks, slices;
  int ntiles_total = 0, nlblk_total = 0, nslice_total = 0, lds_fwd = 0, lds_adj = 0;
  int gv = 0;  // col2im gather variant of the adjoint launches
  int lp_rb = 2;  // row blocks per reduced-precision forward unit
  bool dirty = true;
  bool direct = false;  // launch every round directly (no graph capture or instantiation)
  hipGraphExec_t gexec = nullptr;
  int graph_rounds = 0;
  // graphs of run_aligned: (precision of the rounds, number of rounds) -> graph
  std::map<std::pair<int, int>, hipGraphExec_t> kgraphs;
  // graphs of run_kinds: the precisions launched in each round of a chunk -> graph
  std::map<std::vector<int>, hipGraphExec_t> pgraphs;
  // stage timing (events around each launch) when profiling is on
  struct Prof {
    bool on = false;
    double ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // [4 * (reduced-precision round) + stage]
    int64_t n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    std::vector<hipEvent_t> ev;
  };
  Prof* prof = nullptr;

  Group(Budget* b, const int kdim[3], int prec_, int cap) : budget(b), prec(prec_), capacity(cap) {
    for (int d = 0; d < 3; ++d) kdt[d] = kdim[d];
    contraction_dims(kdt, prec, kd);
    k = kd[0] * kd[1] * kd[2];
    kt = kdt[0] * kdt[1] * kdt[2];
    kp = padded_k(k);
    nsg = (kp + kGroup - 1) / kGroup;
    ncg = nsg;
    states.ensure(budget, sizeof(InstState) * capacity);
    for (int i = capacity - 1; i >= 0; --i) free_slots.push_back(i);
  }
  ~Group() { drop_graph(); }  // prof belongs to the context
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    graph_rounds = 0;
    for (auto& kv : kgraphs) (void)hipGraphExecDestroy(kv.second);
    kgraphs.clear();
    for (auto& kv : pgraphs) (void)hipGraphExecDestroy(kv.second);
    pgraphs.clear();
  }

  void set_v(const float* V, hipStream_t st) {
    Vsrc = V;
    if (kt != k) {
      Vpad.ensure(budget, (size_t)k * k * 4);
      launch_pad_v(V, kdt, kd, Vpad.as<float>(), st);
      V = Vpad.as<float>();
    }
    const size_t n = (size_t)kp * kp;
    Vf.ensure(budget, n * 4);
    Va.ensure(budget, n * 4);
    Vp.ensure(budget, n * 4);
    if (prec != kFP32) {
      Vlo_f.ensure(budget, n * 2);
      Vlo_a.ensure(budget, n * 2);
      Vlo_p.ensure(budget, n * 2);
    }
    launch_prep_v(V, k, kp, Vf.as<float>(), Va.as<float>(), Vp.as<float>(), Vlo_f.p, Vlo_a.p, Vlo_p.p, prec, st);
    if (prec != kFP32 && kp % kGroup == 0) {  // kp admits the tiled adjoint
      Vx_f.ensure(budget, n * 4);
      Vx_p.ensure(budget, n * 4);
      launch_prep_v_x3(V, k, kp, Vx_f.p, Vx_p.p, st);
    }
    HIPCK(hipGetLastError());
  }

  InstState* state_ptr(int slot) const { return states.as<InstState>() + slot; }

  // carve a member's device arrays and fill its descriptor
  void attach(Member* mb, hipStream_t st) {
    if (free_slots.empty()) throw Error(ICNNM_E_BUDGET, "no free slot in group");
    const Plan& p = mb->plan;
    mb->buf.ensure(budget, member_bytes(p, kp, prec));
    char* base = mb->buf.as<char>();
    size_t off = 0;
    auto take = [&](size_t bytes) {
      void* q = base + off;
      off += align256(bytes);
      return q;
    };
    InstDev& d = mb->dev;
    d = InstDev{};
    for (int i = 0; i < 3; ++i) {
      d.m[i] = p.m[i];
      d.k[i] = p.k[i];
      d.b[i] = p.b[i];
      if (p.b[i] <= 0 || (p.b[i] & (p.b[i] - 1))) throw Error(ICNNM_E_INVALID, "tile extents must be powers of two");
      d.lb[i] = __builtin_ctz((unsigned)p.b[i]);
      d.E[i] = p.E[i];
      d.nt[i] = p.nt[i];
      d.C[i] = p.C[i];
      d.goff[i] = p.goff[i];
    }
    d.ntiles = p.ntiles;
    d.gshift = p.gshift;
    d.bm = p.bm;
    d.E123 = p.E123;
    d.nlblk = p.nlblk;
    d.nslice = p.nslice;
    d.mtot = p.mtot;
    d.max_iter = mb->params.max_iter;
    d.refresh_every = mb->params.refresh_every;
    d.prec = prec;
    d.lam = std::isinf(mb->params.lambda) ? 1e308 : mb->params.lambda;
    d.rho = mb->params.rho;
    d.theta_max = mb->params.theta_max;
    d.tol = mb->params.tol;
    d.theta0 = mb->params.theta0;
    d.M = mb->M;
    d.mask = mb->mask;
    d.L = mb->Lout;
    const size_t stf = (size_t)p.ntiles * p.bm * kp;
    d.W = (float*)take(stf * 4);
    d.U = take(stf * (prec != kFP32 ? 2 : 4));
    d.part = (float*)take((size_t)p.ntiles * plan_groups(p, kp) * p.E123 * 4);
    d.qpart = (float*)take((size_t)p.ntiles * kp * 4);
    d.wpart = (float*)take((size_t)p.ntiles * kp * 4);
    d.rpart = (float*)take((size_t)p.ntiles * plan_groups(p, kp) * 4);
    d.dlpart = (double*)take((size_t)p.nlblk * 16);
    d.slice = (double*)take((size_t)(2 * kColRanges * kp + 3 * p.nslice) * 8);
    d.s = (float*)take((size_t)kp * 4);
    int32_t* gt = (int32_t*)take(p.gtab.size() * 4);
    d.gtab = gt;
    if (prec != kFP32) {
      d.D = (float*)take((size_t)p.mtot * 4);
      d.T = (float*)take((size_t)p.mtot * 4);
    }
    HIPCK(hipMemcpyAsync(gt, p.gtab.data(), p.gtab.size() * 4, hipMemcpyHostToDevice, st));
    mb->slot = free_slots.back();
    free_slots.pop_back();
    d.st = state_ptr(mb->slot);
    InstState s0{};
    s0.theta = mb->params.theta0 > 0 ? mb->params.theta0 : -1.0;
    s0.phase = kNew;
    HIPCK(hipMemcpyAsync(d.st, &s0, sizeof(s0), hipMemcpyHostToDevice, st));
    HIPCK(hipStreamSynchronize(st));  // the host sources above are short-lived
    members.push_back(mb);
    dirty = true;
  }

  void detach(Member* mb) {
    auto it = std::find(members.begin(), members.end(), mb);
    if (it != members.end()) members.erase(it);
    if (mb->slot >= 0) free_slots.push_back(mb->slot);
    mb->slot = -1;
    mb->buf.reset();
    dirty = true;
  }

  // rebuild the descriptor array and the tile / L-step / slice tables
  void rebuild(hipStream_t st) {
    std::vector<InstDev> ds;
    std::vector<int2> tl, lb, sl;
    lds_fwd = lds_adj = lds_fwd_x3 = 0;
    gv = members.empty() ? 0 : 8;
    big = kp % kGroup == 0;
    lp_rb = members.empty() ? 2 : 4;
    split = !members.empty();
    for (const Member* mb : members)
      if (!mb->plan.split) split = false;
    for (size_t i = 0; i < members.size(); ++i) {
      const Member* mb = members[i];
      if (!lines_gather_fits(mb->plan)) gv = 0;
      if (mb->plan.bm != 128) big = false;
      if (mb->plan.bm % 128 != 0) lp_rb = 2;
      ds.push_back(mb->dev);
      for (int t = 0; t < mb->plan.ntiles; ++t) tl.push_back(make_int2((int)i, t));
      for (int t = 0; t < mb->plan.nlblk; ++t) lb.push_back(make_int2((int)i, t));
      for (int t = 0; t < mb->plan.nslice; ++t) sl.push_back(make_int2((int)i, t));
      lds_fwd = std::max(lds_fwd, lds_forward_floats(mb->plan, kp, split));
      lds_adj = std::max(lds_adj, lds_adjoint_floats(mb->plan, kp, split));
      lds_fwd_x3 = std::max(lds_fwd_x3, lds_forward_floats(mb->plan, kp, false, true));
    }
    rx3 = prec != kFP32 && big && !members.empty() && lds_fwd_x3 * 4 <= 150 * 1024 &&
          adjoint_big_x3_lds_bytes(kp) <= 160 * 1024 && Vx_f.p != nullptr;
    if (const char* e = getenv("ICNNM_REFRESH"))
      if (strcmp(e, "fp32") == 0) rx3 = false;
    // ICNNM_GATHER=generic keeps the position-owning gather everywhere (compares the
    // two gathers; every plan's box fits both)
    if (const char* e = getenv("ICNNM_GATHER"))
      if (strcmp(e, "generic") == 0) gv = 0;
    // ICNNM_LP_RB=2 keeps 64-row units in the reduced-precision forward (compares the
    // two unit shapes; identical results)
    if (const char* e = getenv("ICNNM_LP_RB"))
      if (atoi(e) == 2) lp_rb = 2;
    ntiles_total = (int)tl.size();
    nlblk_total = (int)lb.size();
    nslice_total = (int)sl.size();
    auto up = [&](DevBuf& b, const void* src, size_t bytes) {
      if (bytes == 0) return;
      if (bytes > b.n) {
        // keep the old buffer until queued work that reads it has finished
        HIPCK(hipStreamSynchronize(st));
        b.ensure(budget, bytes * 2);
      }
      HIPCK(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, st));
    };
    up(inst, ds.data(), ds.size() * sizeof(InstDev));
    up(tiles, tl.data(), tl.size() * sizeof(int2));
    up(lblocks, lb.data(), lb.size() * sizeof(int2));
    up(slices, sl.data(), sl.size() * sizeof(int2));
    HIPCK(hipStreamSynchronize(st));  // host tables go out of scope
    drop_graph();
    dirty = false;
  }

  StageArgs args() const {
    StageArgs a{};
    a.inst = inst.as<InstDev>();
    a.tiles = tiles.as<int2>();
    a.lblocks = lblocks.as<int2>();
    a.slices = slices.as<int2>();
    a.Vf = Vf.as<float>();
    a.Va = Va.as<float>();
    a.Vp = Vp.as<float>();
    a.Vf_lo = Vlo_f.p;
    a.Va_lo = Vlo_a.p;
    a.Vp_lo = Vlo_p.p;
    a.Vf_x = Vx_f.p;
    a.Vp_x = Vx_p.p;
    a.rx3 = rx3 ? 1 : 0;
    a.kp = kp;
    a.k = k;
    a.kt = kt;
    a.u16 = prec != kFP32 ? 1 : 0;
    a.split = split ? 1 : 0;
    a.nsg = split ? kp / kColUnit : nsg;
    a.ncg = split ? kp / kColUnit : ncg;
    a.ntiles = ntiles_total;
    a.tiles_per_slice = kTilesPerSlice;
    a.prec = prec;
    return a;
  }

  // FP32 adjoint (initialisation, FP32 solves, refresh iterations) and, for the reduced
  // precisions, the delta adjoint; each returns at once for instances it does not serve
  // only < 0: both precisions' kernels (each returns at once for the iterations of the
  // other); otherwise only the kernels of precision `only`
  void launch_adjoints(const StageArgs& a, hipStream_t st, int only = -1) const {
    const bool f32 = only < 0 || only == kFP32, lo = prec != kFP32 && (only < 0 || only == prec);
    if (big) {
      // (with rx3 the FP32 adjoint would serve no instance of this reduced-precision group)
      if (f32) launch_adjoint_big(a, ntiles_total, rx3 ? kX3 : kFP32, gv, st);
      if (lo) launch_adjoint_big(a, ntiles_total, prec, gv, st);
    } else {
      if (f32) launch_adjoint(a, ntiles_total, lds_adj, kFP32, gv, st);
      if (lo) launch_adjoint(a, ntiles_total, lds_adj, prec, gv, st);
    }
  }

  void launch_round(hipStream_t st, int only = -1) {
    const StageArgs a = args();
    const bool f32 = only < 0 || only == kFP32, lo = prec != kFP32 && (only < 0 || only == prec);
    launch_colnorm(a, nslice_total, (int)members.size(), st);
    launch_adjoints(a, st, only);
    launch_lstep(a, nlblk_total, st);
    launch_forwards(a, st, f32, lo);
  }

  // FP32 forward (with rx3 only the initialisation), the split-BF16 refresh forward,
  // the reduced-precision delta forward
  void launch_forwards(const StageArgs& a, hipStream_t st, bool f32, bool lo) const {
    if (f32) launch_forward(a, ntiles_total, lds_fwd, kFP32, 2, st);
    if (f32 && rx3) launch_forward(a, ntiles_total, lds_fwd_x3, kX3, 2, st);
    if (lo) launch_forward(a, ntiles_total, lds_fwd, prec, lp_rb, st);
  }

  // one round (launching the precisions `only` selects, as launch_round) with an event
  // pair around each stage; returns after the events are read. Rounds that launch only
  // the reduced-precision contractions are accounted apart from the others.
  void launch_round_timed(hipStream_t st, int only = -1) {
    const StageArgs a = args();
    const bool f32 = only < 0 || only == kFP32, lo = prec != kFP32 && (only < 0 || only == prec);
    if (prof->ev.empty()) {
      prof->ev.resize(8);
      for (auto& e : prof->ev) HIPCK(hipEventCreate(&e));
    }
    HIPCK(hipEventRecord(prof->ev[0], st));
    launch_colnorm(a, nslice_total, (int)members.size(), st);
    HIPCK(hipEventRecord(prof->ev[1], st));
    HIPCK(hipEventRecord(prof->ev[2], st));
    launch_adjoints(a, st, only);
    HIPCK(hipEventRecord(prof->ev[3], st));
    HIPCK(hipEventRecord(prof->ev[4], st));
    launch_lstep(a, nlblk_total, st);
    HIPCK(hipEventRecord(prof->ev[5], st));
    HIPCK(hipEventRecord(prof->ev[6], st));
    launch_forwards(a, st, f32, lo);
    HIPCK(hipEventRecord(prof->ev[7], st));
    HIPCK(hipEventSynchronize(prof->ev[7]));
    const int base = (lo && !f32) ? 4 : 0;
    for (int i = 0; i < 4; ++i) {
      float t = 0;
      HIPCK(hipEventElapsedTime(&t, prof->ev[2 * i], prof->ev[2 * i + 1]));
      prof->ms[base + i] += t;
      prof->n[base + i] += 1;
    }
  }

  // run `rounds` rounds, replaying a captured graph of `chunk` rounds when asked
  void run(int rounds, hipStream_t st, bool use_graph, int chunk) {
    if (dirty) rebuild(st);
    if (members.empty() || rounds <= 0) return;
    if (prof && prof->on) {
      for (int r = 0; r < rounds; ++r) launch_round_timed(st);
      HIPCK(hipGetLastError());
      return;
    }
    if (!use_graph || direct) {
      for (int r = 0; r < rounds; ++r) launch_round(st);
      HIPCK(hipGetLastError());
      return;
    }
    chunk = std::max(1, std::min(chunk, rounds));
    if (!gexec || graph_rounds != chunk) {
      drop_graph();
      hipGraph_t g;
      HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      for (int r = 0; r < chunk; ++r) launch_round(st);
      HIPCK(hipStreamEndCapture(st, &g));
      HIPCK(hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0));
      HIPCK(hipGraphDestroy(g));
      graph_rounds = chunk;
    }
    int done = 0;
    while (done + chunk <= rounds) {
      HIPCK(hipGraphLaunch(gexec, st));
      done += chunk;
    }
    for (; done < rounds; ++done) launch_round(st);
    HIPCK(hipGetLastError());
  }

  // Rounds [r0, r0 + rounds) of a solve whose members all started at round 0 with the
  // same max_iter and refresh_every (single and batch solves): round 0 runs the FP32
  // initial forward, round r >= 1 iteration r, in FP32 when (r - 1) is a multiple of
  // refresh_every or r >= max_iter (the refresh schedule of the column-norm kernel),
  // in the reduced precision otherwise. The host therefore launches only the kernels
  // of each round's precision; a kernel of the other precision would return at once,
  // but its launch still costs several microseconds. Runs of rounds replay cached
  // graphs. FP32 solves take run().
  void run_aligned(int r0, int rounds, hipStream_t st, int max_iter, int refresh_every) {
    if (prec == kFP32) {
      run(rounds, st, true, std::min(std::max(rounds, 1), 16));
      return;
    }
    if (dirty) rebuild(st);
    if (members.empty() || rounds <= 0) return;
    auto kind = [&](int r) { return round_kind(r, prec, max_iter, refresh_every); };
    int r = r0;
    const int end = r0 + rounds;
    if (prof && prof->on) {
      for (; r < end; ++r) launch_round_timed(st, kind(r));
      HIPCK(hipGetLastError());
      return;
    }
    if (direct) {
      for (; r < end; ++r) launch_round(st, kind(r));
      HIPCK(hipGetLastError());
      return;
    }
    while (r < end) {
      const int kd = kind(r);
      int n = 1;
      while (r + n < end && kind(r + n) == kd && n < 16) ++n;
      auto key = std::make_pair(kd, n);
      auto it = kgraphs.find(key);
      if (it == kgraphs.end()) {
        hipGraph_t g;
        hipGraphExec_t ge;
        HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < n; ++i) launch_round(st, kd);
        HIPCK(hipStreamEndCapture(st, &g));
        HIPCK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        HIPCK(hipGraphDestroy(g));
        it = kgraphs.emplace(key, ge).first;
      }
      HIPCK(hipGraphLaunch(it->second, st));
      r += n;
    }
    HIPCK(hipGetLastError());
  }

  // Rounds whose launched precisions are given per round (kinds[r]: kFP32 or the
  // reduced precision alone, or -1 for both), replayed from graphs cached per chunk
  // pattern. Used by the server, whose members sit at different iterations: a round
  // launches only the precisions some member needs in it.
  void run_kinds(const std::vector<int>& kinds, hipStream_t st, int chunk) {
    if (dirty) rebuild(st);
    if (members.empty() || kinds.empty()) return;
    chunk = std::max(1, chunk);
    for (size_t r = 0; r < kinds.size();) {
      const size_t n = std::min(kinds.size() - r, (size_t)chunk);
      std::vector<int> key(kinds.begin() + r, kinds.begin() + r + n);
      auto it = pgraphs.find(key);
      if (it == pgraphs.end()) {
        hipGraph_t g;
        hipGraphExec_t ge;
        HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int kd : key) launch_round(st, kd);
        HIPCK(hipStreamEndCapture(st, &g));
        HIPCK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        HIPCK(hipGraphDestroy(g));
        it = pgraphs.emplace(key, ge).first;
      }
      HIPCK(hipGraphLaunch(it->second, st));
      r += n;
    }
    HIPCK(hipGetLastError());
  }

  void read_states(std::vector<InstState>& out, hipStream_t st) {
    out.resize(capacity);
    HIPCK(hipMemcpyAsync(out.data(), states.p, sizeof(InstState) * capacity, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
  }
};

static void fill_info(const InstState& s, icnnm_info* info) {
  if (!info) return;
  info->iters = s.iters;
  info->converged = s.converged;
  info->r_primal = s.r_primal;
  info->r_change = s.r_change;
  info->objective = s.objective;
  info->theta_final = s.theta;
}

// ------------------------------------------------------------------------------ context
struct Request {
  uint64_t ticket;
  icnnm_shape shape;
  int m[3], kd[3];
  const float* M;
  const uint8_t* mask;
  const float* V;
  icnnm_params params;
  float* Lout;
  double t_submit;
  size_t bytes;        // the member's state and its share of the group's tables
  size_t group_bytes;  // a new group's V operand copies and state array
  int bypassed;        // times later requests were admitted past this one at the head
};

struct Done {
  icnnm_status status;
  icnnm_info info;
};

}  // namespace icnnm

struct icnnm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  icnnm::Budget budget;
  std::recursive_mutex mu;  // serialises synchronous calls
  std::string last_error;
  std::mutex err_mu;
  // cached single-instance groups keyed by (shape, kernel, precision)
  std::map<std::string, std::unique_ptr<icnnm::Group>> cache;
  std::map<std::string, std::unique_ptr<icnnm::Member>> cache_members;
  // serving
  std::mutex q_mu;
  std::condition_variable q_cv;
  std::list<icnnm::Request> queue;
  std::map<uint64_t, icnnm::Done> done;
  std::map<uint64_t, int> pending;  // 1 = queued or running
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread server;
  icnnm::Group::Prof prof;  // stage timing of synchronous calls
  // autotuned tile boxes by (shape, kernel, precision); loaded once from the cache file
  std::map<std::string, std::array<int, 3>> tuned;
  bool tuned_loaded = false;
  // device address of this device's allocation-free scratch (nullptr if unavailable)
  char* scratch = nullptr;
  std::string scratch_err;
};

namespace icnnm {

static void set_error(icnnm_ctx* c, const std::string& m) {
  if (!c) return;
  std::lock_guard<std::mutex> g(c->err_mu);
  c->last_error = m;
}

template <class F>
static icnnm_status guarded(icnnm_ctx* c, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_error(c, e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_error(c, e.what());
    return ICNNM_E_DEVICE;
  } catch (...) {
    set_error(c, "unknown error");
    return ICNNM_E_DEVICE;
  }
}

static void normalize_shape(const icnnm_shape* s, int m[3], int kd[3]) {
  if (!s) throw Error(ICNNM_E_INVALID, "shape is NULL");
  if (s->ndim < 1 || s->ndim > 3) throw Error(ICNNM_E_INVALID, "ndim must be 1, 2 or 3");
  const int lead = 3 - s->ndim;
  for (int d = 0; d < 3; ++d) {
    m[d] = 1;
    kd[d] = 1;
  }
  for (int d = 0; d < s->ndim; ++d) {
    if (s->m[d] < 1 || s->m[d] > (1 << 24)) throw Error(ICNNM_E_INVALID, "tensor dimension out of range");
    if (s->kdim[d] < 1 || s->kdim[d] > s->m[d])
      throw Error(ICNNM_E_INVALID, "kernel dimension must satisfy 1 <= k_j <= m_j");
    m[lead + d] = (int)s->m[d];
    kd[lead + d] = (int)s->kdim[d];
  }
  const int64_t mt = (int64_t)m[0] * m[1] * m[2];
  if (mt > ((int64_t)1 << 31) - 1) throw Error(ICNNM_E_INVALID, "tensor too large");
  const int64_t k = (int64_t)kd[0] * kd[1] * kd[2];
  if (k > 4096) throw Error(ICNNM_E_INVALID, "kernel size k above 4096 is not supported");
}

static void check_params(const icnnm_params* p) {
  if (!p) throw Error(ICNNM_E_INVALID, "params is NULL");
  if (!(p->lambda > 0)) throw Error(ICNNM_E_INVALID, "lambda must be > 0 (or +inf)");
  if (!(p->rho >= 1.0) || !(p->theta_max > 0)) throw Error(ICNNM_E_INVALID, "rho must be >= 1, theta_max > 0");
  if (p->max_iter < 0) throw Error(ICNNM_E_INVALID, "max_iter must be >= 0");
  if (!(p->tol >= 0)) throw Error(ICNNM_E_INVALID, "tol must be >= 0");
  if (p->precision < 0 || p->precision > 2) throw Error(ICNNM_E_INVALID, "unknown precision");
  if (p->precision != 0 && p->refresh_every < 1) throw Error(ICNNM_E_INVALID, "refresh_every must be >= 1");
}

// the reduced precisions pad the innermost kernel extent to a multiple of 4 (see
// contraction_dims); the padded kernel must still fit the tensor
static void check_precision_shape(const int m[3], const int kd[3], const icnnm_params* p) {
  int kdp[3];
  contraction_dims(kd, p->precision, kdp);
  if (kdp[2] > m[2])
    throw Error(ICNNM_E_INVALID, "BF16/FP16 contractions pad the innermost kernel extent to a multiple of 4 (" +
                                     std::to_string(kdp[2]) + "), which must not exceed the innermost tensor extent (" +
                                     std::to_string(m[2]) + ")");
  if ((int64_t)kdp[0] * kdp[1] * kdp[2] > 4096)
    throw Error(ICNNM_E_INVALID, "padded kernel size above 4096 is not supported");
}

static void check_v(icnnm_ctx* c, const float* V, int k, hipStream_t st) {
  float* dv = nullptr;
  HIPCK(hipMallocAsync((void**)&dv, 4, st));
  HIPCK(hipMemsetAsync(dv, 0, 4, st));
  launch_check_v(V, k, dv, st);
  float h = 0;
  HIPCK(hipMemcpyAsync(&h, dv, 4, hipMemcpyDeviceToHost, st));
  HIPCK(hipFreeAsync(dv, st));
  HIPCK(hipStreamSynchronize(st));
  if (!(h <= 1e-5f)) throw Error(ICNNM_E_INVALID, "V is not orthogonal: max|V^T V - I| = " + std::to_string(h));
  (void)c;
}

// order the context stream after the caller's stream
static hipStream_t enter(icnnm_ctx* c, void* user) {
  hipStream_t us = (hipStream_t)user;
  if (us && us != c->stream) {
    HIPCK(hipEventRecord(c->ev_in, us));
    HIPCK(hipStreamWaitEvent(c->stream, c->ev_in, 0));
  }
  return c->stream;
}

static void leave(icnnm_ctx* c, void* user) {
  hipStream_t us = (hipStream_t)user;
  if (us && us != c->stream) {
    HIPCK(hipEventRecord(c->ev_out, c->stream));
    HIPCK(hipStreamWaitEvent(us, c->ev_out, 0));
  }
  HIPCK(hipStreamSynchronize(c->stream));
}

static std::string key_of(const int m[3], const int kd[3], const icnnm_params* p) {
  char buf[256];
  snprintf(buf, sizeof buf, "%d,%d,%d|%d,%d,%d|%d", m[0], m[1], m[2], kd[0], kd[1], kd[2], p->precision);
  return buf;
}

// ------------------------------------------------------------------------------ autotuner
// With ICNNM_AUTOTUNE=1 the tile box of an instance is chosen by measurement: the
// cost model's kTuneCandidates cheapest boxes each run kTuneRounds solver rounds of
// the actual instance (scratch state and output, after two warm-up iterations) and
// the fastest is kept, per (shape, kernel, precision), for the life of the context
// and, if ICNNM_AUTOTUNE_CACHE names a file, across processes (one line per key:
// "icnnm-tile m0 m1 m2 k0 k1 k2 precision class b0 b1 b2"). Without it the cost
// model decides alone. In a batch the members share kernel variants (the tiled
// adjoint needs 128-row tiles, the line gather line-friendly boxes), so there the
// search keeps to boxes of the cost model's class (same rows per tile, same gather),
// recorded as class 1 in the key. Tile boxes change the summation order of the
// col2im and of the column-norm partials, not the method: results agree to rounding.
constexpr int kTuneCandidates = 4;
constexpr int kTuneRounds = 10;

static bool autotune_on() {
  const char* e = getenv("ICNNM_AUTOTUNE");
  return e && atoi(e) != 0;
}

static std::string tune_key(const int m[3], const int kd[3], int prec, int cls) {
  char buf[128];
  snprintf(buf, sizeof buf, "%d %d %d %d %d %d %d %d", m[0], m[1], m[2], kd[0], kd[1], kd[2], prec, cls);
  return buf;
}

static void load_tune_cache(icnnm_ctx* c) {
  if (c->tuned_loaded) return;
  c->tuned_loaded = true;
  const char* path = getenv("ICNNM_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[256];
  while (fgets(line, sizeof line, f)) {
    int v[11];
    if (sscanf(line, "icnnm-tile %d %d %d %d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5],
               &v[6], &v[7], &v[8], &v[9], &v[10]) == 11)
      c->tuned[tune_key(v, v + 3, v[6], v[7])] = {v[8], v[9], v[10]};
  }
  fclose(f);
}

static void save_tune_entry(const std::string& key, const int b[3]) {
  const char* path = getenv("ICNNM_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "icnnm-tile %s %d %d %d\n", key.c_str(), b[0], b[1], b[2]);
  fclose(f);
}

// seconds per solver round of one instance under plan p
static double time_plan(icnnm_ctx* c, const Plan& p, const int kd[3], int prec, const float* M,
                        const uint8_t* mask, const float* V, hipStream_t st) {
  DevBuf Ls;
  Ls.ensure(&c->budget, (size_t)p.mtot * 4);
  Group g(&c->budget, kd, prec, 1);
  Member mb;
  mb.plan = p;
  icnnm_params_default(&mb.params);
  mb.params.precision = prec;
  mb.params.max_iter = 1 << 20;
  mb.M = M;
  mb.mask = mask;
  mb.Lout = Ls.as<float>();
  struct Events {  // destroyed on every exit path
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  HIPCK(hipEventCreate(&ev.e[0]));
  HIPCK(hipEventCreate(&ev.e[1]));
  g.attach(&mb, st);
  g.set_v(V, st);
  g.run(4, st, false, 1);  // new -> init -> two iterations
  HIPCK(hipEventRecord(ev.e[0], st));
  g.run(kTuneRounds, st, false, 1);
  HIPCK(hipEventRecord(ev.e[1], st));
  HIPCK(hipEventSynchronize(ev.e[1]));
  float ms = 0.f;
  HIPCK(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
  g.detach(&mb);
  return 1e-3 * ms / kTuneRounds;
}

// tile plan of an instance: measured (autotuner) or the cost model's
static Plan choose_plan(icnnm_ctx* c, const int m[3], const int kd[3], int kp, int prec, const float* M,
                        const uint8_t* mask, const float* V, hipStream_t st, bool same_class,
                        bool may_measure = true) {
  int kdp[3];
  contraction_dims(kd, prec, kdp);
  // an instance solved alone may take the split contractions; members of joint
  // launches never do
  auto split_of = [&](Plan p) {
    if (!same_class) decide_split(p, kp, prec);
    return p;
  };
  auto base_plan = [&] { return split_of(same_class ? make_plan_shared(m, kdp, kp) : make_plan(m, kdp, kp)); };
  if (!autotune_on() || getenv("ICNNM_TILE")) return base_plan();
  load_tune_cache(c);
  const std::string key = tune_key(m, kd, prec, same_class ? 1 : 0);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) return split_of(plan_with_box(m, kdp, kp, it->second.data()));
  if (!may_measure) return base_plan();
  auto all = plan_candidates(m, kdp, kp);
  if (all.empty()) throw Error(ICNNM_E_INVALID, "no tile shape fits this problem");
  std::vector<Plan> cands;
  const Plan first = base_plan();
  for (auto& cp : all) {
    if ((int)cands.size() == kTuneCandidates) break;
    if (same_class && (cp.second.bm != first.bm || lines_gather_fits(cp.second) != lines_gather_fits(first)))
      continue;
    cands.push_back(cp.second);
  }
  int best = 0;
  double best_t = 1e300;
  for (int i = 0; i < (int)cands.size(); ++i) {
    Plan p = cands[i];
    finish_plan(p, kp);
    p = split_of(p);
    double t = 1e300;
    try {
      t = time_plan(c, p, kd, prec, M, mask, V, st);
    } catch (const Error& e) {
      // a candidate whose state does not fit the budget is skipped; any other error
      // is the solve's own
      if (e.code != ICNNM_E_BUDGET && e.code != ICNNM_E_NOMEM) throw;
      HIPCK(hipStreamSynchronize(st));
    }
    if (t < best_t) {
      best_t = t;
      best = i;
    }
  }
  if (best_t >= 1e300) return base_plan();  // nothing could be timed
  Plan p = cands[best];
  finish_plan(p, kp);
  p = split_of(p);
  c->tuned[key] = {p.b[0], p.b[1], p.b[2]};
  save_tune_entry(key, p.b);
  return p;
}

static void fill_tile(const Plan& p, icnnm_info* info) {
  if (!info) return;
  for (int d = 0; d < 3; ++d) info->tile[d] = p.b[d];
  info->split = p.split ? 1 : 0;
}

static icnnm_status do_solve(icnnm_ctx* c, const icnnm_shape* shape, const float* M, const uint8_t* mask,
                             const float* V, const icnnm_params* params, float* L_out, icnnm_info* info,
                             void* user_stream) {
  int m[3], kd[3];
  normalize_shape(shape, m, kd);
  check_params(params);
  check_precision_shape(m, kd, params);
  if (!M || !mask || !V || !L_out) throw Error(ICNNM_E_INVALID, "NULL array argument");
  std::lock_guard<std::recursive_mutex> lock(c->mu);
  hipStream_t st = enter(c, user_stream);
  const int k = kd[0] * kd[1] * kd[2];
  if (params->check_v) check_v(c, V, k, st);
  const std::string key = key_of(m, kd, params);
  auto it = c->cache.find(key);
  Group* g;
  Member* mb;
  if (it == c->cache.end()) {
    auto grp = std::make_unique<Group>(&c->budget, kd, params->precision, 1);
    auto mem = std::make_unique<Member>();
    mem->plan = choose_plan(c, m, kd, grp->kp, params->precision, M, mask, V, st, false);
    mem->params = *params;
    mem->M = M;
    mem->mask = mask;
    mem->Lout = L_out;
    grp->attach(mem.get(), st);
    g = grp.get();
    mb = mem.get();
    c->cache[key] = std::move(grp);
    c->cache_members[key] = std::move(mem);
  } else {
    g = it->second.get();
    mb = c->cache_members[key].get();
    // re-point the descriptor at this call's arrays and reset the state
    mb->params = *params;
    mb->M = M;
    mb->mask = mask;
    mb->Lout = L_out;
    InstDev& d = mb->dev;
    d.M = M;
    d.mask = mask;
    d.L = L_out;
    d.max_iter = params->max_iter;
    d.refresh_every = params->refresh_every;
    d.lam = std::isinf(params->lambda) ? 1e308 : params->lambda;
    d.rho = params->rho;
    d.theta_max = params->theta_max;
    d.tol = params->tol;
    d.theta0 = params->theta0;
    InstState s0{};
    s0.theta = params->theta0 > 0 ? params->theta0 : -1.0;
    s0.phase = kNew;
    HIPCK(hipMemcpyAsync(d.st, &s0, sizeof(s0), hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(g->inst.p, &d, sizeof(InstDev), hipMemcpyHostToDevice, st));
    HIPCK(hipStreamSynchronize(st));
  }
  g->set_v(V, st);
  g->prof = &c->prof;
  const double t0 = now_s();
  const int total = params->max_iter + 2;  // new -> init, init -> first iteration, final reduction
  if (params->tol > 0) {
    int ran = 0;
    std::vector<InstState> sts;
    while (ran < total) {
      const int chunk = std::min(10, total - ran);
      g->run_aligned(ran, chunk, st, params->max_iter, params->refresh_every);
      ran += chunk;
      g->read_states(sts, st);
      if (sts[mb->slot].phase == kDone) break;
    }
  } else {
    g->run_aligned(0, total, st, params->max_iter, params->refresh_every);
  }
  std::vector<InstState> sts;
  g->read_states(sts, st);
  leave(c, user_stream);
  const InstState& s = sts[mb->slot];
  if (info) {
    fill_info(s, info);
    fill_tile(mb->plan, info);
    info->refresh_x3 = g->rx3 ? 1 : 0;
    info->t_queue_s = 0;
    info->t_device_s = now_s() - t0;
  }
  if (s.phase != kDone) throw Error(ICNNM_E_DEVICE, "solver did not reach its final state");
  if (s.status != 0) {
    set_error(c, "NaN or Inf in a residual");
    return ICNNM_E_NUMERIC;
  }
  return ICNNM_OK;
}

static icnnm_status do_solve_batch(icnnm_ctx* c, int count, const icnnm_shape* shapes, const float* const* Ms,
                                   const uint8_t* const* masks, const float* V, const icnnm_params* params,
                                   float* const* Louts, icnnm_info* infos, void* user_stream) {
  if (count < 0 || (count > 0 && (!shapes || !Ms || !masks || !Louts || !V)))
    throw Error(ICNNM_E_INVALID, "bad batch arguments");
  check_params(params);
  if (count == 0) return ICNNM_OK;
  int kd0[3];
  std::vector<std::unique_ptr<Member>> mems;
  for (int i = 0; i < count; ++i) {
    int m[3], kd[3];
    normalize_shape(&shapes[i], m, kd);
    if (i == 0) std::copy(kd, kd + 3, kd0);
    check_precision_shape(m, kd, params);
    if (!std::equal(kd, kd + 3, kd0)) throw Error(ICNNM_E_INVALID, "batch instances must share the kernel size");
    if (!Ms[i] || !masks[i] || !Louts[i]) throw Error(ICNNM_E_INVALID, "NULL array in batch");
    auto mb = std::make_unique<Member>();
    mb->params = *params;
    mb->M = Ms[i];
    mb->mask = masks[i];
    mb->Lout = Louts[i];
    mems.push_back(std::move(mb));
    (void)m;
  }
  std::lock_guard<std::recursive_mutex> lock(c->mu);
  hipStream_t st = enter(c, user_stream);
  Group g(&c->budget, kd0, params->precision, count);
  if (params->check_v) check_v(c, V, g.kt, st);
  for (int i = 0; i < count; ++i) {
    int m[3], kd[3];
    normalize_shape(&shapes[i], m, kd);
    mems[i]->plan = choose_plan(c, m, kd, g.kp, params->precision, Ms[i], masks[i], V, st, true);
    g.attach(mems[i].get(), st);
  }
  g.set_v(V, st);
  g.prof = &c->prof;
  const double t0 = now_s();
  const int total = params->max_iter + 2;
  if (params->tol > 0) {
    int ran = 0;
    std::vector<InstState> sts;
    while (ran < total) {
      const int chunk = std::min(10, total - ran);
      g.run_aligned(ran, chunk, st, params->max_iter, params->refresh_every);
      ran += chunk;
      g.read_states(sts, st);
      bool all = true;
      for (auto& mb : mems) all = all && sts[mb->slot].phase == kDone;
      if (all) break;
    }
  } else {
    g.run_aligned(0, total, st, params->max_iter, params->refresh_every);
  }
  std::vector<InstState> sts;
  g.read_states(sts, st);
  leave(c, user_stream);
  icnnm_status rc = ICNNM_OK;
  for (int i = 0; i < count; ++i) {
    const InstState& s = sts[mems[i]->slot];
    if (infos) {
      fill_info(s, &infos[i]);
      fill_tile(mems[i]->plan, &infos[i]);
      infos[i].refresh_x3 = g.rx3 ? 1 : 0;
      infos[i].t_queue_s = 0;
      infos[i].t_device_s = now_s() - t0;
    }
    if (s.status != 0) rc = ICNNM_E_NUMERIC;
    if (s.phase != kDone) rc = ICNNM_E_DEVICE;
  }
  for (auto& mb : mems) g.detach(mb.get());
  g.prof = nullptr;
  if (rc != ICNNM_OK) set_error(c, "one or more batch instances failed");
  return rc;
}

// ------------------------------------------------------------------------------ allocation-free solve
// Scratch of icnnm_solve_noalloc: every device array the solver needs beyond the
// caller's inputs and output (V operand layouts, instance state, multiplier and Z-step
// operand, halo partials, reduction slices, gather and tile tables) is carved from this
// array, so the call makes no device allocation. Each device holds its own copy (from
// module load to process end); in host code the name is only a handle: its device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocBytes = (size_t)160 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// device address of `scratch` on the current device, looked up once per device
static char* scratch_address(int device, std::string& err) {
  static std::mutex mu;
  static std::map<int, char*> addr;
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return nullptr;
  }
  addr[device] = (char*)ptr;
  return (char*)ptr;
}

// one allocation-free call at a time per device in this process: they share its scratch
static std::mutex& scratch_lock(int device) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<std::mutex>> locks;
  std::lock_guard<std::mutex> g(mu);
  auto& l = locks[device];
  if (!l) l = std::make_unique<std::mutex>();
  return *l;
}

// bytes of the scratch a solve of plan p takes (bump order of do_solve_noalloc)
static size_t noalloc_bytes(const Plan& p, int kp, int prec) {
  size_t b = 256;                                                   // check_v result
  b += align256(sizeof(InstState));                                  // state slot
  b += align256(member_bytes(p, kp, prec));                          // instance state
  b += 3 * align256((size_t)kp * kp * 4);                            // V layouts (FP32)
  if (prec != kFP32) b += 3 * align256((size_t)kp * kp * 2);         // V layouts (16-bit)
  if (prec != kFP32 && kp % kGroup == 0) b += 2 * align256((size_t)kp * kp * 4);  // split-BF16 V
  b += align256(2 * sizeof(InstDev)) + 3 * align256(2 * 8 * ((size_t)p.ntiles + p.nlblk + p.nslice));  // tables
  return b;
}

static icnnm_status do_solve_noalloc(icnnm_ctx* c, const icnnm_shape* shape, const float* M, const uint8_t* mask,
                                     const float* V, const icnnm_params* params, float* L_out, icnnm_info* info,
                                     void* user_stream) {
  int m[3], kd[3];
  normalize_shape(shape, m, kd);
  check_params(params);
  check_precision_shape(m, kd, params);
  if (!M || !mask || !V || !L_out) throw Error(ICNNM_E_INVALID, "NULL array argument");
  if (!c->scratch) throw Error(ICNNM_E_DEVICE, "allocation-free scratch unavailable: " + c->scratch_err);
  const int k = kd[0] * kd[1] * kd[2];
  int kdp[3];
  contraction_dims(kd, params->precision, kdp);
  const int kc = kdp[0] * kdp[1] * kdp[2];
  const int kp = padded_k(kc);
  Budget arena;  // outlives every buffer carved from it
  arena.arena = c->scratch;
  arena.limit = kNoAllocBytes;
  Member mb;
  mb.plan = make_plan(m, kdp, kp);  // the cost model's box (no measurement: it would allocate)
  decide_split(mb.plan, kp, params->precision);
  const size_t need = noalloc_bytes(mb.plan, kp, params->precision) + (kc != k ? (size_t)kc * kc * 4 + 256 : 0);
  if (need > kNoAllocBytes)
    throw Error(ICNNM_E_BUDGET, "instance needs " + std::to_string(need) + " bytes of solver state, above the " +
                                    std::to_string(kNoAllocBytes >> 20) + " MiB allocation-free scratch maximum");
  std::lock_guard<std::recursive_mutex> lock(c->mu);
  std::lock_guard<std::mutex> slock(scratch_lock(c->device));
  hipStream_t st = enter(c, user_stream);
  if (params->check_v) {
    float* dv = (float*)arena.alloc(256);
    launch_fill_f32(dv, 0.f, 1, st);  // the scratch keeps the previous call's contents
    launch_check_v(V, k, dv, st);
    float h = 0.f;
    HIPCK(hipMemcpyAsync(&h, dv, 4, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (!(h <= 1e-5f)) throw Error(ICNNM_E_INVALID, "V is not orthogonal: max|V^T V - I| = " + std::to_string(h));
  }
  {
    Group g(&arena, kd, params->precision, 1);
    g.direct = true;
    mb.params = *params;
    mb.M = M;
    mb.mask = mask;
    mb.Lout = L_out;
    // every device array is written before it is read (the descriptor and state are
    // uploaded, the first forward writes U and Q of every tile row, ragged rows
    // included), so nothing left in the scratch by an earlier call is used
    g.attach(&mb, st);
    g.set_v(V, st);
    const double t0 = now_s();
    const int total = params->max_iter + 2;
    std::vector<InstState> sts;
    if (params->tol > 0) {
      int ran = 0;
      while (ran < total) {
        const int chunk = std::min(10, total - ran);
        g.run_aligned(ran, chunk, st, params->max_iter, params->refresh_every);
        ran += chunk;
        g.read_states(sts, st);
        if (sts[mb.slot].phase == kDone) break;
      }
    } else {
      g.run_aligned(0, total, st, params->max_iter, params->refresh_every);
    }
    g.read_states(sts, st);
    leave(c, user_stream);
    const InstState& s = sts[mb.slot];
    if (info) {
      fill_info(s, info);
      fill_tile(mb.plan, info);
      info->refresh_x3 = g.rx3 ? 1 : 0;
      info->t_queue_s = 0;
      info->t_device_s = now_s() - t0;
    }
    g.detach(&mb);
    if (s.phase != kDone) throw Error(ICNNM_E_DEVICE, "solver did not reach its final state");
    if (s.status != 0) {
      set_error(c, "NaN or Inf in a residual");
      return ICNNM_E_NUMERIC;
    }
  }
  return ICNNM_OK;
}

// ------------------------------------------------------------------------------ learning
// Eigen-decomposition of the k x k FP64 Gram G (device) by the parallel cyclic Jacobi
// kernels (jacobi.hip): w descending, V row-major [s][i] with column i the eigenvector
// of w[i], its largest-magnitude entry made positive (the first of equal ones). An odd
// k gets a zero row and column appended: that index never rotates (its off-diagonal
// entries are zero), so its eigenvector stays the unit vector and is dropped.
static void device_eig(Budget* bud, const double* G, int k, hipStream_t st, std::vector<double>& w,
                       std::vector<double>& V) {
  const int n = k + (k & 1);
  const size_t nn = (size_t)n * n;
  DevBuf A0, A1, V0, V1, nrm, rot;
  A0.ensure(bud, nn * 8);
  A1.ensure(bud, nn * 8);
  V0.ensure(bud, nn * 8);
  V1.ensure(bud, nn * 8);
  nrm.ensure(bud, (2 + 512) * 8);
  rot.ensure(bud, (size_t)3 * (n / 2 + 1) * 8);
  launch_jacobi_init(G, k, A0.as<double>(), V0.as<double>(), n, st);
  double *A = A0.as<double>(), *B = A1.as<double>(), *Vc = V0.as<double>(), *W = V1.as<double>();
  bool converged = n <= 1;
  for (int sweep = 0; sweep < 40 && !converged; ++sweep) {
    for (int r = 0; r + 1 < n; ++r) {
      launch_jacobi_round(A, B, Vc, W, n, rot.as<double>(), st);
      std::swap(A, B);
      std::swap(Vc, W);
    }
    HIPCK(hipGetLastError());
    launch_jacobi_offnorm(A, n, nrm.as<double>() + 2, nrm.as<double>(), st);
    double h[2] = {0.0, 0.0};
    HIPCK(hipMemcpyAsync(h, nrm.p, 16, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (!std::isfinite(h[0]) || !std::isfinite(h[1])) throw Error(ICNNM_E_NUMERIC, "NaN or Inf in the Gram matrix");
    converged = h[0] <= 1e-28 * h[1];  // off-diagonal Frobenius norm <= 1e-14 of the whole
  }
  if (!converged) throw Error(ICNNM_E_NUMERIC, "Jacobi eigensolver did not converge");
  std::vector<double> Ah(nn), Vh(nn);
  HIPCK(hipMemcpyAsync(Ah.data(), A, nn * 8, hipMemcpyDeviceToHost, st));
  HIPCK(hipMemcpyAsync(Vh.data(), Vc, nn * 8, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  std::vector<int> cols;
  for (int c = 0; c < n; ++c)
    if (n == k || Vh[(size_t)k * n + c] == 0.0) cols.push_back(c);
  if ((int)cols.size() != k) throw Error(ICNNM_E_NUMERIC, "Jacobi eigensolver lost the padding index");
  std::stable_sort(cols.begin(), cols.end(),
                   [&](int a, int b) { return Ah[(size_t)a * n + a] > Ah[(size_t)b * n + b]; });
  w.assign(k, 0.0);
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) {
    const int c = cols[i];
    w[i] = Ah[(size_t)c * n + c];
    int arg = 0;
    double best = -1.0;
    for (int s = 0; s < k; ++s) {
      const double v = std::fabs(Vh[(size_t)s * n + c]);
      if (v > best) {
        best = v;
        arg = s;
      }
    }
    const double sg = Vh[(size_t)arg * n + c] < 0 ? -1.0 : 1.0;
    for (int s = 0; s < k; ++s) V[(size_t)s * k + i] = sg * Vh[(size_t)s * n + c];
  }
}

static icnnm_status do_learn(icnnm_ctx* c, const int64_t kdim_in[3], int b, const icnnm_shape* shapes,
                             const float* const* refs, float* V_out, double* eig_out, void* user_stream) {
  if (b < 1 || !shapes || !refs || !V_out || !kdim_in) throw Error(ICNNM_E_INVALID, "bad learn arguments");
  const int nd = shapes[0].ndim;
  icnnm_shape ks = shapes[0];
  for (int d = 0; d < nd; ++d) ks.kdim[d] = kdim_in[d];
  int m0[3], kd[3];
  normalize_shape(&ks, m0, kd);
  const int k = kd[0] * kd[1] * kd[2];
  std::lock_guard<std::recursive_mutex> lock(c->mu);
  hipStream_t st = enter(c, user_stream);
  const int ndiff = (2 * kd[0] - 1) * (2 * kd[1] - 1) * (2 * kd[2] - 1);
  DevBuf R, G, part;
  R.ensure(&c->budget, (size_t)ndiff * 8);
  G.ensure(&c->budget, (size_t)k * k * 8);
  part.ensure(&c->budget, autocorr_part_doubles(kd) * 8);
  HIPCK(hipMemsetAsync(R.p, 0, (size_t)ndiff * 8, st));
  for (int j = 0; j < b; ++j) {
    icnnm_shape sj = shapes[j];
    if (sj.ndim != nd) throw Error(ICNNM_E_INVALID, "reference tensors must share the order");
    for (int d = 0; d < nd; ++d) sj.kdim[d] = kdim_in[d];
    int m[3], kk[3];
    normalize_shape(&sj, m, kk);
    if (!refs[j]) throw Error(ICNNM_E_INVALID, "NULL reference");
    launch_autocorr(refs[j], m, kd, R.as<double>(), part.as<double>(), st);
  }
  launch_gram_expand(R.as<double>(), kd, G.as<double>(), st);
  HIPCK(hipGetLastError());
  std::vector<double> w, Vd;
  device_eig(&c->budget, G.as<double>(), k, st, w, Vd);
  std::vector<float> Vf(Vd.size());
  for (size_t i = 0; i < Vd.size(); ++i) Vf[i] = (float)Vd[i];
  HIPCK(hipMemcpyAsync(V_out, Vf.data(), Vf.size() * 4, hipMemcpyHostToDevice, st));
  leave(c, user_stream);
  if (eig_out) std::copy(w.begin(), w.end(), eig_out);
  return ICNNM_OK;
}

// Diagnostics of L0 under V (Definition 2, eq:rkL0, eq:alphaK): the Gram of A_k(L0)
// from circular autocorrelations (as in learning), C = V^T G V on the device in FP64,
// sigma_i = sqrt(C_ii), r_K = #{sigma_i > rtol max sigma}, alpha_K^2 = the largest
// eigenvalue of D C D with D = diag(1 / sigma_i) on the support.
static icnnm_status do_diag(icnnm_ctx* c, const icnnm_shape* shape, const float* L0, const float* V, double rtol,
                            double* sigma_out, int32_t* rank_out, double* alpha_out, void* user_stream) {
  if (!L0 || !V) throw Error(ICNNM_E_INVALID, "L0 and V must be device pointers");
  if (!(rtol > 0.0)) throw Error(ICNNM_E_INVALID, "rtol must be positive");
  int m[3], kd[3];
  normalize_shape(shape, m, kd);
  const int k = kd[0] * kd[1] * kd[2];
  std::lock_guard<std::recursive_mutex> lock(c->mu);
  hipStream_t st = enter(c, user_stream);
  const int ndiff = (2 * kd[0] - 1) * (2 * kd[1] - 1) * (2 * kd[2] - 1);
  const size_t kk = (size_t)k * k;
  DevBuf R, G, Vd, T, Cm, part;
  R.ensure(&c->budget, (size_t)ndiff * 8);
  part.ensure(&c->budget, autocorr_part_doubles(kd) * 8);
  G.ensure(&c->budget, kk * 8);
  Vd.ensure(&c->budget, kk * 8);
  T.ensure(&c->budget, kk * 8);
  Cm.ensure(&c->budget, kk * 8);
  HIPCK(hipMemsetAsync(R.p, 0, (size_t)ndiff * 8, st));
  launch_autocorr(L0, m, kd, R.as<double>(), part.as<double>(), st);
  launch_gram_expand(R.as<double>(), kd, G.as<double>(), st);
  launch_f32_to_f64(V, Vd.as<double>(), (int64_t)kk, st);
  launch_gemm_f64(G.as<double>(), 0, Vd.as<double>(), T.as<double>(), k, st);   // T = G V
  launch_gemm_f64(Vd.as<double>(), 1, T.as<double>(), Cm.as<double>(), k, st);  // C = V^T T
  HIPCK(hipGetLastError());
  std::vector<double> Ch(kk);
  HIPCK(hipMemcpyAsync(Ch.data(), Cm.p, kk * 8, hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  leave(c, user_stream);
  std::vector<double> sig(k);
  double smax = 0.0;
  for (int i = 0; i < k; ++i) {
    sig[i] = std::sqrt(std::max(Ch[(size_t)i * k + i], 0.0));
    smax = std::max(smax, sig[i]);
  }
  const double thr = rtol * std::max(smax, 1e-300);
  std::vector<double> d(k, 0.0);
  int rank = 0;
  for (int i = 0; i < k; ++i)
    if (sig[i] > thr) {
      d[i] = 1.0 / sig[i];
      ++rank;
    }
  double alpha = 0.0;
  if (alpha_out) {
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) Ch[(size_t)i * k + j] *= d[i] * d[j];
    std::vector<double> w, Vv;
    sym_eig(Ch, k, w, Vv);
    alpha = std::sqrt(std::max(w.empty() ? 0.0 : w[0], 0.0));
  }
  if (sigma_out) std::copy(sig.begin(), sig.end(), sigma_out);
  if (rank_out) *rank_out = rank;
  if (alpha_out) *alpha_out = alpha;
  return ICNNM_OK;
}

}  // namespace icnnm

// ================================================================================ C ABI
using namespace icnnm;

extern "C" {

void icnnm_params_default(icnnm_params* p) {
  if (!p) return;
  p->lambda = INFINITY;
  p->theta0 = 0.0;
  p->rho = 1.1;
  p->theta_max = 1e10;
  p->max_iter = 100;
  p->tol = 0.0;
  p->precision = ICNNM_PREC_FP32;
  p->refresh_every = 10;
  p->check_v = 0;
}

icnnm_status icnnm_create(int device, size_t hbm_budget_bytes, icnnm_ctx** out) {
  if (!out) return ICNNM_E_INVALID;
  *out = nullptr;
  auto* c = new (std::nothrow) icnnm_ctx();
  if (!c) return ICNNM_E_NOMEM;
  icnnm_status rc = guarded(c, [&]() -> icnnm_status {
    int n = 0;
    HIPCK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) throw Error(ICNNM_E_DEVICE, "no such HIP device");
    HIPCK(hipSetDevice(device));
    c->device = device;
    HIPCK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIPCK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIPCK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    size_t fr = 0, tot = 0;
    HIPCK(hipMemGetInfo(&fr, &tot));
    c->budget.limit = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
    // this device's copy of the allocation-free scratch (looked up once per device)
    c->scratch = scratch_address(device, c->scratch_err);
    return ICNNM_OK;
  });
  if (rc != ICNNM_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return ICNNM_OK;
}

void icnnm_destroy(icnnm_ctx* c);

const char* icnnm_last_error(const icnnm_ctx* c) {
  if (!c) return "NULL context";
  // a per-thread copy: the serving thread may record a new error at any time
  thread_local std::string copy;
  {
    std::lock_guard<std::mutex> g(const_cast<icnnm_ctx*>(c)->err_mu);
    copy = c->last_error;
  }
  return copy.c_str();
}

icnnm_status icnnm_learn_eigvecs(icnnm_ctx* c, const int64_t kdim[3], int32_t b, const icnnm_shape ref_shapes[],
                                 const float* const refs[], float* V_out, double* eigvals_out, void* stream) {
  if (!c) return ICNNM_E_INVALID;
  return guarded(c, [&] { return do_learn(c, kdim, b, ref_shapes, refs, V_out, eigvals_out, stream); });
}

icnnm_status icnnm_diagnostics(icnnm_ctx* c, const icnnm_shape* shape, const float* L0, const float* V, double rtol,
                               double* sigma_out, int32_t* rank_out, double* alpha_out, void* stream) {
  if (!c) return ICNNM_E_INVALID;
  return guarded(c, [&] { return do_diag(c, shape, L0, V, rtol, sigma_out, rank_out, alpha_out, stream); });
}

icnnm_status icnnm_solve(icnnm_ctx* c, const icnnm_shape* shape, const float* M, const uint8_t* mask,
                         const float* V, const icnnm_params* params, float* L_out, icnnm_info* info,
                         void* stream) {
  if (!c) return ICNNM_E_INVALID;
  return guarded(c, [&] { return do_solve(c, shape, M, mask, V, params, L_out, info, stream); });
}

icnnm_status icnnm_plan(const icnnm_shape* shape, const icnnm_params* params, int32_t joint, icnnm_plan_info* out) {
  if (!shape || !params || !out) return ICNNM_E_INVALID;
  try {
    int m[3], kd[3];
    normalize_shape(shape, m, kd);
    check_params(params);
    check_precision_shape(m, kd, params);
    int kdp[3];
    contraction_dims(kd, params->precision, kdp);
    const int kp = padded_k(kdp[0] * kdp[1] * kdp[2]);
    Plan p = joint ? make_plan_shared(m, kdp, kp) : make_plan(m, kdp, kp);
    if (!joint) decide_split(p, kp, params->precision);
    for (int d = 0; d < 3; ++d) {
      out->tile[d] = p.b[d];
      out->tiles_per_dim[d] = p.nt[d];
    }
    out->ntiles = p.ntiles;
    out->padded_k = kp;
    out->state_bytes = (int64_t)member_bytes(p, kp, params->precision);
    out->split = p.split ? 1 : 0;
    return ICNNM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return ICNNM_E_INVALID;
  }
}

icnnm_status icnnm_solve_noalloc(icnnm_ctx* c, const icnnm_shape* shape, const float* M, const uint8_t* mask,
                                 const float* V, const icnnm_params* params, float* L_out, icnnm_info* info,
                                 void* stream) {
  if (!c) return ICNNM_E_INVALID;
  return guarded(c, [&] { return do_solve_noalloc(c, shape, M, mask, V, params, L_out, info, stream); });
}

icnnm_status icnnm_solve_batch(icnnm_ctx* c, int32_t count, const icnnm_shape shapes[], const float* const M[],
                               const uint8_t* const masks[], const float* V, const icnnm_params* params,
                               float* const L_out[], icnnm_info infos[], void* stream) {
  if (!c) return ICNNM_E_INVALID;
  return guarded(c, [&] { return do_solve_batch(c, count, shapes, M, masks, V, params, L_out, infos, stream); });
}

}  // extern "C"

// ================================================================================ serving
namespace icnnm {

// Requests that share V, kernel size and precision iterate in one group; each group
// has its own stream, so groups of different kernel sizes overlap on the device.
struct ServeGroup {
  std::unique_ptr<Group> g;
  std::vector<std::unique_ptr<Member>> active;
  hipStream_t stream = nullptr;
  std::vector<InstState> sts;
  double work = 0.0;  // sum over members of m kp^2: the cost of one round
  ServeGroup() = default;
  ServeGroup(const ServeGroup&) = delete;
  ServeGroup& operator=(const ServeGroup&) = delete;
  ~ServeGroup() {
    g.reset();
    if (stream) (void)hipStreamDestroy(stream);
  }
};

static std::string group_key(const float* V, const int kd[3], int prec) {
  char buf[160];
  snprintf(buf, sizeof buf, "%p|%d,%d,%d|%d", (const void*)V, kd[0], kd[1], kd[2], prec);
  return buf;
}

constexpr int kServeSlots = 512;
constexpr int kServeRounds = 4;      // rounds per scheduling pass of the costliest group
constexpr int kServeMaxRounds = 64;  // ... and at most for cheaper groups
constexpr int kBypassScan = 16;      // queued requests looked at past a blocked head
constexpr int kMaxBypass = 32;       // admissions past one blocked head before strict FIFO

// Releases the single-instance solve cache (state of earlier icnnm_solve calls kept for
// reuse), whose budget share can otherwise block a served request indefinitely. Takes
// the synchronous-call lock, so it waits for a solve in flight on another thread.
static void evict_solve_cache(icnnm_ctx* c) {
  std::lock_guard<std::recursive_mutex> lock(c->mu);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  c->cache_members.clear();
  c->cache.clear();
}

// Continuous batching: admit queued requests while the HBM budget allows, run all
// admitted requests of a (V, kernel, precision) group in joint launches, retire
// finished ones after each chunk of rounds.
static void serve_loop(icnnm_ctx* c) {
  (void)hipSetDevice(c->device);
  std::map<std::string, ServeGroup> groups;
  bool evicted = false;  // the solve cache was released for a blocked head
  for (;;) {
    std::vector<Request> admit;
    bool any_active = false;
    bool head_blocked = false;
    {
      std::unique_lock<std::mutex> lk(c->q_mu);
      for (auto& kv : groups) any_active = any_active || !kv.second.active.empty();
      if (!any_active) c->q_cv.wait(lk, [&] { return c->stop || !c->queue.empty(); });
      if (c->stop && c->queue.empty() && !any_active) break;
      // Admission (admission_pass): cumulative reservation within the pass, a new
      // group's bytes with its first request, at most kServeSlots members per group,
      // bounded bypass of a blocked head.
      std::vector<AdmitView> views;
      std::vector<std::list<Request>::iterator> where;
      for (auto it = c->queue.begin(); it != c->queue.end(); ++it) {
        views.push_back(AdmitView{group_key(it->V, it->kd, it->params.precision), it->bytes, it->group_bytes, &it->bypassed});
        where.push_back(it);
      }
      std::map<std::string, int> free_slots;
      for (auto& kv : groups)
        if (kv.second.g) free_slots[kv.first] = (int)kv.second.g->free_slots.size();
      const AdmitResult ar = admission_pass(
          views, free_slots, AdmitLimits{c->budget.used.load(), c->budget.limit, kServeSlots, kMaxBypass, kBypassScan});
      for (size_t i : ar.admitted) {
        admit.push_back(*where[i]);
        c->queue.erase(where[i]);
      }
      head_blocked = ar.head_blocked;
    }
    if (admit.empty() && head_blocked && !any_active) {
      // Nothing runs and the head does not fit: budget is held outside the server.
      // Release the solve cache once; if the head still cannot be admitted with
      // nothing else holding budget, it never will (submit checks the request alone
      // against the whole budget, so this is a safety net): fail it.
      if (!evicted) {
        evict_solve_cache(c);
        evicted = true;
        continue;
      }
      std::lock_guard<std::mutex> lk(c->q_mu);
      Request r = c->queue.front();
      c->queue.pop_front();
      set_error(c, "request does not fit the HBM budget with nothing else admitted");
      Done d{};
      d.status = ICNNM_E_BUDGET;
      c->done[r.ticket] = d;
      c->pending.erase(r.ticket);
      evicted = false;
      continue;
    }
    if (!admit.empty()) evicted = false;
    std::vector<Request> requeue;
    for (Request& r : admit) {
      icnnm_status rc = guarded(c, [&]() -> icnnm_status {
        const std::string key = group_key(r.V, r.kd, r.params.precision);
        ServeGroup& sg = groups[key];
        if (!sg.g) {
          HIPCK(hipStreamCreateWithFlags(&sg.stream, hipStreamNonBlocking));
          sg.g = std::make_unique<Group>(&c->budget, r.kd, r.params.precision, kServeSlots);
          sg.g->set_v(r.V, sg.stream);
        }
        auto mb = std::make_unique<Member>();
        mb->plan = make_plan_shared(r.m, sg.g->kd, sg.g->kp);
        mb->params = r.params;
        mb->M = r.M;
        mb->mask = r.mask;
        mb->Lout = r.Lout;
        mb->ticket = r.ticket;
        mb->t_submit = r.t_submit;
        mb->t_start = now_s();
        sg.g->attach(mb.get(), sg.stream);
        sg.work += (double)mb->plan.mtot * sg.g->kp * sg.g->kp;
        sg.active.push_back(std::move(mb));
        return ICNNM_OK;
      });
      if (rc == ICNNM_E_BUDGET || rc == ICNNM_E_NOMEM) {
        // budget taken meanwhile by a synchronous call on another thread: queue again
        requeue.push_back(r);
      } else if (rc != ICNNM_OK) {
        std::lock_guard<std::mutex> lk(c->q_mu);
        Done d{};
        d.status = rc;
        c->done[r.ticket] = d;
        c->pending.erase(r.ticket);
      }
    }
    if (!requeue.empty()) {
      std::lock_guard<std::mutex> lk(c->q_mu);
      for (auto it = requeue.rbegin(); it != requeue.rend(); ++it) c->queue.push_front(*it);
    }
    for (auto it = groups.begin(); it != groups.end();) {
      if (it->second.active.empty())
        it = groups.erase(it);
      else
        ++it;
    }
    // launch every group's rounds on its own stream first, then collect: groups run
    // concurrently, and a cheaper group runs proportionally more rounds per pass so
    // that its requests are not held back by the rounds of a costlier group. Members
    // know their refresh schedule, so each round launches only the contraction
    // precisions that some member needs in it.
    double wmax = 0.0;
    for (auto& kv : groups) wmax = std::max(wmax, kv.second.work);
    std::map<std::string, icnnm_status> rcs;
    for (auto& kv : groups) {
      ServeGroup& sg = kv.second;
      const double share = sg.work > 0.0 ? wmax / sg.work : 1.0;
      const int rounds = (int)std::min<double>(kServeMaxRounds, kServeRounds * std::max(1.0, std::floor(share)));
      // per chunk of kServeRounds rounds: only FP32, only the reduced precision, or
      // both (a chunk is uniform, so a group keeps at most three cached graphs, which
      // matters because membership changes drop them)
      std::vector<int> kinds(rounds, kFP32);
      if (sg.g->prec != kFP32) {
        for (int r0 = 0; r0 < rounds; r0 += kServeRounds) {
          bool f32 = false, lo = false;
          for (int r = r0; r < std::min(rounds, r0 + kServeRounds); ++r)
            for (auto& mb : sg.active) {
              const int kd = round_kind(mb->round + r, sg.g->prec, mb->params.max_iter, mb->params.refresh_every);
              (kd == kFP32 ? f32 : lo) = true;
            }
          const int kd = f32 && lo ? -1 : (f32 ? (int)kFP32 : sg.g->prec);
          for (int r = r0; r < std::min(rounds, r0 + kServeRounds); ++r) kinds[r] = kd;
        }
      }
      rcs[kv.first] = guarded(c, [&]() -> icnnm_status {
        sg.g->run_kinds(kinds, sg.stream, kServeRounds);
        return ICNNM_OK;
      });
      for (auto& mb : sg.active) mb->round += rounds;
    }
    for (auto& kv : groups) {
      ServeGroup& sg = kv.second;
      icnnm_status rc = rcs[kv.first];
      if (rc == ICNNM_OK) rc = guarded(c, [&]() -> icnnm_status {
        sg.g->read_states(sg.sts, sg.stream);
        return ICNNM_OK;
      });
      std::vector<std::unique_ptr<Member>> keep;
      for (auto& mb : sg.active) {
        const InstState* s = rc == ICNNM_OK ? &sg.sts[mb->slot] : nullptr;
        if (s && s->phase != kDone) {
          keep.push_back(std::move(mb));
          continue;
        }
        Done d{};
        d.status = rc != ICNNM_OK ? rc : (s->status != 0 ? ICNNM_E_NUMERIC : ICNNM_OK);
        if (s) fill_info(*s, &d.info);
        fill_tile(mb->plan, &d.info);
        d.info.refresh_x3 = sg.g->rx3 ? 1 : 0;
        const double t = now_s();
        d.info.t_queue_s = mb->t_start - mb->t_submit;
        d.info.t_device_s = t - mb->t_start;
        sg.work -= (double)mb->plan.mtot * sg.g->kp * sg.g->kp;
        sg.g->detach(mb.get());
        std::lock_guard<std::mutex> lk(c->q_mu);
        c->done[mb->ticket] = d;
        c->pending.erase(mb->ticket);
      }
      sg.active = std::move(keep);
    }
  }
}

static icnnm_status do_submit(icnnm_ctx* c, const icnnm_shape* shape, const float* M, const uint8_t* mask,
                              const float* V, const icnnm_params* params, float* L_out, uint64_t* ticket) {
  if (!ticket) throw Error(ICNNM_E_INVALID, "ticket is NULL");
  Request r{};
  normalize_shape(shape, r.m, r.kd);
  check_params(params);
  check_precision_shape(r.m, r.kd, params);
  if (!M || !mask || !V || !L_out) throw Error(ICNNM_E_INVALID, "NULL array argument");
  r.shape = *shape;
  r.M = M;
  r.mask = mask;
  r.V = V;
  r.params = *params;
  r.Lout = L_out;
  r.t_submit = now_s();
  const int k = r.kd[0] * r.kd[1] * r.kd[2];
  int kdp[3];
  contraction_dims(r.kd, params->precision, kdp);
  const int kc = kdp[0] * kdp[1] * kdp[2];
  const int kp = padded_k(kc);
  const Plan p = make_plan_shared(r.m, kdp, kp);  // as the server will plan it
  // the member's state, plus its entries in the group's descriptor and tile tables
  // (which grow by doubling)
  r.bytes = member_bytes(p, kp, params->precision) +
            2 * align256(sizeof(InstDev) + 8 * ((size_t)p.ntiles + p.nlblk + p.nslice));
  // a new group: V operand copies (three FP32 layouts, three more in BF16/FP16 for the
  // reduced precisions, and the two split-BF16 ones where kp admits the tiled adjoint)
  // and the state array of its slots
  r.group_bytes = align256((size_t)kp * kp * 4) * 3 + (params->precision != 0 ? 3 * align256((size_t)kp * kp * 2) : 0) +
                  (params->precision != 0 && kp % kGroup == 0 ? 2 * align256((size_t)kp * kp * 4) : 0) +
                  align256(sizeof(InstState) * kServeSlots) + (kc != k ? align256((size_t)kc * kc * 4) : 0);
  r.bypassed = 0;
  if (r.bytes + r.group_bytes > c->budget.limit) throw Error(ICNNM_E_BUDGET, "request alone exceeds the HBM budget");
  if (params->check_v) {
    // checked before the request is queued, on the context's stream
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    check_v(c, V, k, c->stream);
  }
  std::lock_guard<std::mutex> lk(c->q_mu);
  if (!c->server.joinable()) c->server = std::thread(serve_loop, c);
  r.ticket = c->next_ticket++;
  c->pending[r.ticket] = 1;
  c->queue.push_back(r);
  *ticket = r.ticket;
  c->q_cv.notify_one();
  return ICNNM_OK;
}

static icnnm_status do_poll(icnnm_ctx* c, uint64_t ticket, icnnm_info* info) {
  std::lock_guard<std::mutex> lk(c->q_mu);
  if (c->pending.count(ticket)) return ICNNM_PENDING;
  auto it = c->done.find(ticket);
  if (it == c->done.end()) throw Error(ICNNM_E_NOTFOUND, "unknown ticket");
  if (info) *info = it->second.info;
  const icnnm_status rc = it->second.status;
  c->done.erase(it);
  return rc;
}

}  // namespace icnnm

extern "C" {

icnnm_status icnnm_submit(icnnm_ctx* c, const icnnm_shape* shape, const float* M, const uint8_t* mask,
                          const float* V, const icnnm_params* params, float* L_out, uint64_t* ticket) {
  if (!c) return ICNNM_E_INVALID;
  return guarded(c, [&] { return do_submit(c, shape, M, mask, V, params, L_out, ticket); });
}

icnnm_status icnnm_poll(icnnm_ctx* c, uint64_t ticket, icnnm_info* info) {
  if (!c) return ICNNM_E_INVALID;
  return guarded(c, [&] { return do_poll(c, ticket, info); });
}

icnnm_status icnnm_set_profiling(icnnm_ctx* c, int32_t enable) {
  if (!c) return ICNNM_E_INVALID;
  std::lock_guard<std::recursive_mutex> lock(c->mu);
  c->prof.on = enable != 0;
  return ICNNM_OK;
}

icnnm_status icnnm_stage_times(icnnm_ctx* c, double ms[8], int64_t counts[8], int32_t reset) {
  if (!c || !ms || !counts) return ICNNM_E_INVALID;
  std::lock_guard<std::recursive_mutex> lock(c->mu);
  for (int i = 0; i < 8; ++i) {
    ms[i] = c->prof.ms[i];
    counts[i] = c->prof.n[i];
    if (reset) {
      c->prof.ms[i] = 0;
      c->prof.n[i] = 0;
    }
  }
  return ICNNM_OK;
}

void icnnm_destroy(icnnm_ctx* c) {
  if (!c) return;
  {
    std::lock_guard<std::mutex> lk(c->q_mu);
    c->stop = true;
  }
  c->q_cv.notify_all();
  if (c->server.joinable()) c->server.join();
  {
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    c->cache_members.clear();
    c->cache.clear();
    for (auto& e : c->prof.ev) (void)hipEventDestroy(e);
    c->prof.ev.clear();
  }
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"

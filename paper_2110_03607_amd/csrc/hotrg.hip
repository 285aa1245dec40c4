// Host engine and C ABI of libhotrg.so (declared in include/hotrg.h).
//
// One coarse-graining step along the Current direction (Sections 3-4 of the paper),
// everything enqueued on the caller's stream:
//   1. Gram matrices A^(j), A'^(j) in three steps (Section 3.2): permute T so that the
//      (side leg, c') or (side leg, c) pair is the row index, FP64 MFMA GEMM X X^T with
//      split-K and a fixed-order reduction, then the (rho, eta) contraction.
//   2. FP64 eigendecomposition of A and A' (Householder tridiagonalisation, Sturm bisection,
//      inverse iteration; Section 4.2.5).
//   3. Judgement values, choice, truncation (Sections 2, 4.2.6-4.2.7).
//   4. For each chunk of new-tensor columns (the paper's loop over n'_1, Section 4.2.9):
//      prime chain -> B operand, bottleneck GEMM on MFMA in the precision form,
//      non-prime chain + renaming into T^next.
//   5. Trace, Gu-Wen ratio, lnZ/V, normalisation (Sections 4.1.1, 4.2.11, 4.2.15-4.2.17).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hotrg.h"
#include "kernels.h"

using namespace hk;

namespace {

constexpr long TILE_M = 256, TILE_N = 256, TILE_K = 64;   // operand padding (multiple of every tile)
constexpr long GRAM_TILE = 128;                             // tile of the FP64 Gram GEMM
constexpr int MAX_CHI_3D = 16, MAX_CHI_2D = 32;
// 4D: the register width of the 4D chain kernels (every chi_j, k_j <= 12), and element counts of
// order H^2 = chi^8 that stay within 32-bit indices.
constexpr int MAX_CHI_4D = 12;
inline int max_chi_for(int d, int) { return d == 2 ? MAX_CHI_2D : d == 3 ? MAX_CHI_3D : MAX_CHI_4D; }
// register width of the 4D chain kernels for these dims (8 when every chi_j and k_j is at most 8)
inline int cn4_for(const Dims& dm) {
  const int m = std::max(std::max(std::max(dm.chi1, dm.chi2), std::max(dm.chi3, dm.k1)), std::max(dm.k2, dm.k3));
  return m <= 8 ? 8 : 12;
}
constexpr size_t ALIGN = 256;
constexpr int EIG_SLOTS = EIG_BATCH;   // (direction, side) matrices decomposed per step, at most

inline long roundup(long x, long m) { return (x + m - 1) / m * m; }

bool form_valid(int f) { return f >= HOTRG_FP64 && f <= HOTRG_SPLIT_FP16; }
size_t master_size(int form) { return form == HOTRG_FP64 ? 8 : 4; }
size_t op_esize(int form) {
  switch (form) {
    case HOTRG_FP64: return 8;
    case HOTRG_FP32: return 4;
    default: return 2;
  }
}
int op_planes(int form) { return (form == HOTRG_SPLIT_BF16 || form == HOTRG_SPLIT_FP16) ? 2 : 1; }
size_t acc_size(int form) { return form == HOTRG_FP64 ? 8 : 4; }

// Dimensions of the current tensor: slot 0 = c, slot j = n_j.
struct LocalDims {
  int d;
  int chi[MAXD];
};

Dims make_dims(const LocalDims& ld, const int* k) {
  Dims dm;
  dm.d = ld.d;
  dm.chic = ld.chi[0];
  dm.chi1 = ld.chi[1];
  dm.chi2 = ld.d >= 3 ? ld.chi[2] : 1;
  dm.chi3 = ld.d >= 4 ? ld.chi[3] : 1;
  dm.k1 = k[0];
  dm.k2 = ld.d >= 3 ? k[1] : 1;
  dm.k3 = ld.d >= 4 ? k[2] : 1;
  dm.b = dm.chi1 * dm.chi2 * dm.chi3;
  dm.H = dm.chic * dm.b;
  return dm;
}

// Gram GEMM geometry for one side of one direction.
struct GramGeo {
  long R, Rp, C, Cp, kchunk;
  int Z;
};
GramGeo gram_geo(long H, long R) {
  GramGeo g;
  g.R = R;
  // R <= 64 (3D chi = 8, 4D): 64 x 64 tiles, so that no padding rows are read or multiplied
  const long tile = R <= 64 ? 64 : GRAM_TILE;
  g.Rp = roundup(R, tile);
  g.C = H * H / R;
  const long tiles = (g.Rp / tile) * (g.Rp / tile);
  long Z = std::max(1L, (512 + tiles - 1) / tiles);
  Z = std::min(Z, std::max(1L, roundup(g.C, 16) / 16));
  g.kchunk = roundup((g.C + Z - 1) / Z, tile == 64 ? 32 : 16);   // a multiple of the GEMM's K step
  g.Z = (int)((g.C + g.kchunk - 1) / g.kchunk);
  g.Cp = (long)g.Z * g.kchunk;
  return g;
}

// Byte sizes of every workspace region for given dims (max over the run is allocated).
struct Need {
  size_t T, Aop, Bop, Cc, X, part, G, Amat, w, Ut, comb, W2;
};

// The third Gram step as a GEMM (large directions): P[(fh, gh)][(r, e)] from Gh, Q likewise
// from Gc, S = P Q^T, then A[fh + chi fc][gh + chi gc] = S[(fh, gh)][(fc, gc)].
constexpr long COMB_GEMM_N = 512;
struct CombGeo {
  long n, Mp, Kp;
};
inline CombGeo comb_geo(long chis, long chic) {
  CombGeo c;
  c.n = chis * chis;
  c.Mp = roundup(c.n, 128);
  c.Kp = roundup(chic * chic, 16);
  return c;
}

// Derivative mode doubles the operand rows ([dT | T] and [C2 | dC2]) and the product chunk.
inline int grad_mult(bool grad) { return grad ? 2 : 1; }

long chunk_pairs_for(const LocalDims& ld, const int* k, int form, int user_chunk, bool grad = false) {
  long total = 1;
  for (int j = 1; j < ld.d; ++j) total *= k[j - 1];
  if (user_chunk > 0) return std::min<long>(total, user_chunk);
  const Dims dm = make_dims(ld, k);
  const long Kp = roundup(dm.H, TILE_K), Mp = roundup(dm.H, TILE_M);
  const double per_pair = (double)dm.chic * dm.b * (Kp * op_esize(form) * op_planes(form) + Mp * acc_size(form)) *
                          grad_mult(grad);
  const double budget = 2.0 * 1024 * 1024 * 1024;
  long c = (long)std::max(1.0, std::floor(budget / per_pair));
  return std::min(total, c);
}

Need need_for(const LocalDims& ld, int chi, int form, int user_chunk, bool grad = false) {
  Need n{};
  int k[MAXD];
  for (int j = 1; j < ld.d; ++j) k[j - 1] = std::min(ld.chi[j] * ld.chi[j], chi);
  const Dims dm = make_dims(ld, k);
  const long H = dm.H;
  const long Mp = roundup(H, TILE_M), Kp = roundup(H, TILE_K);
  const long pairs = chunk_pairs_for(ld, k, form, user_chunk, grad);
  const long Np = roundup(pairs * dm.chic * dm.b, TILE_N);
  long Hn = dm.chic;
  for (int j = 0; j < ld.d - 1; ++j) Hn *= k[j];
  n.T = (size_t)std::max(H * H, Hn * Hn) * master_size(form);
  n.Aop = (size_t)Mp * Kp * op_esize(form) * op_planes(form) * grad_mult(grad);
  n.Bop = (size_t)Np * Kp * op_esize(form) * op_planes(form) * grad_mult(grad);
  n.Cc = (size_t)Mp * Np * acc_size(form);
  // 4D non-prime chain scratch: W2[(c, g)][(nh1, nc1)][(n2, n3)] of one chunk (8-byte elements)
  if (ld.d == 4)
    n.W2 = (size_t)pairs * dm.chic * dm.chic * dm.chi1 * dm.chi1 * dm.k2 * dm.k3 * 8;
  size_t X = 0, part = 0, G = 0, Am = 0;
  for (int j = 1; j < ld.d; ++j) {
    const GramGeo g = gram_geo(H, (long)ld.chi[j] * ld.chi[0]);
    X = std::max(X, (size_t)(g.Rp * g.Cp) * 8);
    part = std::max(part, (size_t)g.Z * g.Rp * g.Rp * 8);
    G = std::max(G, (size_t)g.R * g.R * 8);
    const long nn = (long)ld.chi[j] * ld.chi[j];
    Am = std::max(Am, (size_t)nn * nn * 8);
    if (nn >= COMB_GEMM_N) {
      const CombGeo cg = comb_geo(ld.chi[j], ld.chi[0]);
      n.comb = std::max(n.comb, (size_t)(2 * cg.Mp * cg.Kp + cg.Mp * cg.Mp) * 8);
    }
  }
  n.X = X;
  n.part = part;
  n.G = G;
  n.Amat = Am;
  n.w = (size_t)chi * chi * 8 + 64;
  n.Ut = (size_t)chi * chi * chi * 8;
  return n;
}

void need_max(Need& a, const Need& b) {
  a.T = std::max(a.T, b.T); a.Aop = std::max(a.Aop, b.Aop); a.Bop = std::max(a.Bop, b.Bop);
  a.Cc = std::max(a.Cc, b.Cc); a.X = std::max(a.X, b.X); a.part = std::max(a.part, b.part);
  a.G = std::max(a.G, b.G); a.Amat = std::max(a.Amat, b.Amat); a.w = std::max(a.w, b.w);
  a.Ut = std::max(a.Ut, b.Ut); a.W2 = std::max(a.W2, b.W2);
  a.comb = std::max(a.comb, b.comb);
}

// All bond dimensions a run can reach from the starting dimensions: each of them, then
// min(x^2, chi) repeatedly.
std::vector<int> reachable_dims(const std::vector<int>& starts, int chi) {
  std::vector<int> v;
  for (int x : starts) {
    for (;;) {
      if (std::find(v.begin(), v.end(), x) == v.end()) v.push_back(x);
      const int nx = std::min(x * x, chi);
      if (nx == x || x >= chi) break;
      x = nx;
    }
  }
  return v;
}

struct Plan {
  Need need;
  size_t off_state, off_rec, off_T, off_Tn, off_Aop, off_Bop, off_Cc, off_X, off_part, off_Gh, off_Gc,
      off_A, off_Vw, off_Vo, off_w, off_Ut, off_Ut32, off_comb, off_W2, total;
  // derivative mode (0 when off)
  size_t off_dT, off_dTn, off_dCc, off_Xd, off_dGh, off_dGc, off_dA, off_dUt, off_dUt32, off_dUw;
  bool grad;
  int max_steps;
};

// Maximum needs over every bond-dimension combination a run can reach.
Need plan_need(int d, const std::vector<int>& starts, int chi, int form, int user_chunk, bool grad) {
  Need nd{};
  const std::vector<int> vals = reachable_dims(starts, chi);
  LocalDims ld;
  ld.d = d;
  const int nv = (int)vals.size();
  int combos = 1;
  for (int i = 0; i < d; ++i) combos *= nv;
  for (int cidx = 0; cidx < combos; ++cidx) {
    int r = cidx;
    for (int i = 0; i < d; ++i) { ld.chi[i] = vals[r % nv]; r /= nv; }
    need_max(nd, need_for(ld, chi, form, user_chunk, grad));
  }
  return nd;
}

inline size_t take_at(size_t& o, size_t bytes) {
  const size_t r = o;
  o = roundup(o + bytes, ALIGN);
  return r;
}

// Regions that hold one run's state from step to step: device state and step records
// (contiguous, cleared at init), the tensor pair, the Gram matrices and eigenvectors, the
// isometries, and the derivative copies.
void place_private(Plan& P, size_t& o, const Need& nd, int max_steps, bool grad) {
  P.off_state = take_at(o, sizeof(DevState));
  P.off_rec = take_at(o, sizeof(StepRec) * (size_t)(max_steps + 1));
  P.off_T = take_at(o, nd.T);
  P.off_Tn = take_at(o, nd.T);
  P.off_A = take_at(o, EIG_SLOTS * nd.Amat);
  P.off_Vw = take_at(o, EIG_SLOTS * 2 * nd.Amat);
  P.off_Vo = take_at(o, EIG_SLOTS * nd.Amat);
  P.off_w = take_at(o, EIG_SLOTS * nd.w);
  P.off_Ut = take_at(o, MAXD * nd.Ut);
  P.off_Ut32 = take_at(o, MAXD * nd.Ut / 2 + 64);
  if (grad) {
    P.off_dT = take_at(o, nd.T);
    P.off_dTn = take_at(o, nd.T);
    P.off_dA = take_at(o, EIG_SLOTS * nd.Amat);
    P.off_dUt = take_at(o, MAXD * nd.Ut);
    P.off_dUt32 = take_at(o, MAXD * nd.Ut / 2 + 64);
  }
}

// Scratch used only inside one step (operands, products, Gram pieces): runs that execute
// one after the other on the same stream may share it.
void place_scratch(Plan& P, size_t& o, const Need& nd, bool grad) {
  P.off_Aop = take_at(o, nd.Aop);
  P.off_Bop = take_at(o, nd.Bop);
  P.off_Cc = take_at(o, nd.Cc);
  P.off_X = take_at(o, nd.X);
  P.off_part = take_at(o, nd.part);
  P.off_Gh = take_at(o, nd.G);
  P.off_Gc = take_at(o, nd.G);
  P.off_comb = take_at(o, nd.comb);
  P.off_W2 = take_at(o, nd.W2);
  if (grad) {
    P.off_dCc = take_at(o, nd.Cc);
    P.off_Xd = take_at(o, nd.X);
    P.off_dGh = take_at(o, nd.G);
    P.off_dGc = take_at(o, nd.G);
    P.off_dUw = take_at(o, 2 * nd.Amat);   // k_dU: W = dA U_kept and the coefficients U^T W
  }
}

Plan make_plan(int d, const std::vector<int>& starts, int chi, int form, int user_chunk, int max_steps,
               bool grad = false) {
  Plan P{};
  const Need nd = plan_need(d, starts, chi, form, user_chunk, grad);
  P.need = nd;
  P.max_steps = max_steps;
  P.grad = grad;
  size_t o = 0;
  place_private(P, o, nd, max_steps, grad);
  place_scratch(P, o, nd, grad);
  P.total = o;
  return P;
}

// Relative rounding of the Gram spectrum in each form (the multiplet floor of k_choose): 16 unit
// roundoffs of the arithmetic that bounds the form's accuracy (0 for FP64: the exact multiplet
// rule of the oracle).  Split FP16 operands carry 22 bits, more than the FP32 master tensor and
// accumulation they feed, so its value is FP32's.
double multiplet_tau(int form) {
  switch (form) {
    case HOTRG_FP64: return 0.0;
    case HOTRG_FP32: return 16.0 * 0x1p-24;
    case HOTRG_SPLIT_FP16: return 16.0 * 0x1p-24;
    case HOTRG_SPLIT_BF16: return 16.0 * 0x1p-16;
    case HOTRG_FP16: return 16.0 * 0x1p-11;
    default: return 16.0 * 0x1p-8;
  }
}

unsigned grid_for(long n, int block = 256) {
  long g = (n + block - 1) / block;
  return (unsigned)std::max(1L, std::min(g, 65536L));
}

// Grid of the kernels that end in one atomic per workgroup on a single device scalar
// (max|T|): a grid-stride loop over at most 1024 workgroups keeps those atomics few.
unsigned grid_reduce(long n) { return std::min(grid_for(n), 1024u); }

// Clears n ints (one workgroup; used instead of a memset so that recorded streams hold kernels only).
__global__ void k_zero_int(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Multi-workgroup tridiagonalisation of the large matrices of an eigensolver batch (one
// launch per reflector); k_eigh_tri then finishes every matrix.
void enqueue_tri_steps(const EigBatch& eb, hipStream_t s) {
  int maxn = 0;
  for (int i = 0; i < eb.count; ++i) maxn = std::max(maxn, eb.n[i]);
  if (maxn < TRI_MULTI_N) return;
  const unsigned gx = (unsigned)((maxn - 1 + TRI_ROWS - 1) / TRI_ROWS);
  for (int st = 0; st < tri_lds_start(maxn); ++st)
    hipLaunchKernelGGL(k_tri_step, dim3(gx, (unsigned)eb.count), dim3(256), 0, s, eb, st);
  hipLaunchKernelGGL(k_tri_finish, dim3((unsigned)eb.count), dim3(EIG_THREADS), 0, s, eb);
}

// After enqueue_tri_steps: eigenpairs of every matrix of eb, by the one-workgroup solver or,
// for the large truncated ones (eig_split), by the split kernels.
void enqueue_eig_finish(const EigBatch& eb, hipStream_t s) {
  int whole = 0, wb = 0, kv = 0;
  for (int i = 0; i < eb.count; ++i) {
    if (eig_split(eb.n[i], eb.kvec[i])) {
      wb = std::max(wb, (eig_nev(eb.n[i], eb.kvec[i]) + EB_EPW - 1) / EB_EPW);
      kv = std::max(kv, eb.kvec[i]);
    } else {
      ++whole;
    }
  }
  if (whole) hipLaunchKernelGGL(k_eigh_tri, dim3((unsigned)eb.count), dim3(EIG_THREADS), 0, s, eb);
  if (wb) {
    hipLaunchKernelGGL(k_eig_bisect, dim3((unsigned)wb, (unsigned)eb.count), dim3(EB_THREADS), 0, s, eb);
    hipLaunchKernelGGL(k_eig_invit, dim3((unsigned)eb.count), dim3(EI_THREADS), 0, s, eb);
    hipLaunchKernelGGL(k_eig_backtr, dim3((unsigned)kv, (unsigned)eb.count), dim3(64), 0, s, eb);
  }
}

}  // namespace

struct hotrg_handle {
  hotrg_model model{};
  hotrg_opts opts{};
  double beta = 0;
  int chi = 0;
  int form = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t s = nullptr;
  Plan plan{};
  LocalDims ld{};
  int axes[MAXD]{};   // lattice axis of each slot (slot 0 = Current)
  int p = 0;
  bool failed = false;
  bool no_fuse = false;   // force the separate non-prime kernel (tests of the fused epilogue)
  bool scalar_prime = false;   // force the one-element-per-thread prime chain (debug contraction)
  // set by the batch autotuner: pair groups per chunk (0: the plan's) and the 128 x 128
  // tile GEMM instead of the 256 x 256 one for the 16-bit forms
  int tune_chunk = 0;
  bool tune_small_tiles = false;
  bool tune_no_f12 = false;   // set by the batch autotuner: 3D chi = 12 through the 256 x 256 GEMM unfused
  bool grad = false;      // derivative mode: carry dT/dbeta through every step
  std::string err;
  // live timing: pairs of events recorded on the stream, resolved at hotrg_timings
  bool profiling = false;
  struct Pending { int cat; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  hotrg_timing acc{};

  template <class X> X* at(size_t off) { return reinterpret_cast<X*>(ws + off); }
  DevState* st() { return at<DevState>(plan.off_state); }
  StepRec* rec(int step) { return at<StepRec>(plan.off_rec) + step; }
};

struct hotrg_batch {
  int n = 0;
  hotrg_opts opts{};
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t s = nullptr;
  std::vector<hotrg_handle*> inst;
  // eigensolver descriptor tables, one per distinct dims signature of a step
  size_t off_tables = 0;
  int table_cap = 0;                       // descriptors per table
  int n_tables = 0;                        // table slots in the workspace
  struct Table { std::vector<EigDesc> key; int slot; };
  std::vector<Table> tables;
  int next_slot = 0;
  // recorded steps: one graph per parity of the step (the tensor buffers alternate)
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  bool use_graphs = true;
  int p = 0;
  int graph_launches = 0, eager_steps = 0;
  struct Tuned { int d, chi, tile, chunk; double ms; };
  std::vector<Tuned> tuned;
  bool failed = false;
  std::string err;
  template <class X> X* at(size_t off) { return reinterpret_cast<X*>(ws + off); }
};

namespace {

thread_local std::string g_static_err;

// Timing helpers: mark(h) records an event on the stream (or returns null when not
// profiling); close(h, cat, start) records the end event and queues the pair.
hipEvent_t tmark(hotrg_handle* h) {
  if (!h->profiling) return nullptr;
  hipEvent_t e;
  if (!h->free_events.empty()) {
    e = h->free_events.back();
    h->free_events.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  if (hipEventRecord(e, h->s) != hipSuccess) {
    h->free_events.push_back(e);
    return nullptr;
  }
  return e;
}
void tclose(hotrg_handle* h, int cat, hipEvent_t start) {
  if (!h->profiling || !start) return;
  hipEvent_t e = tmark(h);
  if (!e) return;
  h->pending.push_back({cat, start, e});
}

int fail(hotrg_handle* h, int code, const std::string& msg) {
  if (h) {
    h->err = msg;
    if (code == HOTRG_E_DEVICE || code == HOTRG_E_NUMERIC) h->failed = true;
  } else {
    g_static_err = msg;
  }
  return code;
}

#define HIPCHK(h, expr)                                                              \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return fail((h), HOTRG_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Launch helpers (template dispatch on the precision form)
// ---------------------------------------------------------------------------

template <int F> struct GemmCfg;
template <> struct GemmCfg<F_FP64> { static constexpr int BK = 16; };
template <> struct GemmCfg<F_FP32> { static constexpr int BK = 32; };
template <> struct GemmCfg<F_BF16> { static constexpr int BK = 64; };
template <> struct GemmCfg<F_FP16> { static constexpr int BK = 64; };
template <> struct GemmCfg<F_SPLIT_BF16> { static constexpr int BK = 64; };
template <> struct GemmCfg<F_SPLIT_FP16> { static constexpr int BK = 64; };

// Operand tiles of the large-tile GEMM loaded straight into LDS (k_gemm_big, DL) for the two-plane
// forms and FP32, where it was measured faster (split FP16 bottleneck 4.76 -> 4.54 ms per launch,
// FP32 16.3 -> 15.7 ms at chi = 16); the single-plane 16-bit forms keep the register staging
// (2.78 ms against 3.01 ms with direct loads).
template <int F> constexpr int gemm_sched() { return (FormInfo<F>::planes == 2 || F == F_FP32) ? 1 : 0; }

template <int F>
void launch_gemm(const void* A, long lda, long aplane, const void* B, long ldb, long bplane, void* C, long ldc,
                 long czs, long Mp, long Np, long Kp, int Z, long kchunk, const double* scale_ptr, double smult,
                 hipStream_t s, const FuseArgs* fuse = nullptr, bool small_tiles = false) {
  typedef typename OpOf<F>::type Op;
  constexpr int PL = FormInfo<F>::planes;
  if constexpr (F != F_FP64) {
    // FP32 goes through the same kernel with four-k fragments (OpF32v)
    typedef typename std::conditional<F == F_FP32, OpF32v, Op>::type OpB;
    if (!small_tiles && Z == 1 && smult == 1.0 && Mp % GB_BM == 0 && Np % GB_BN == 0 && Kp % 64 == 0) {
      const int mt = (int)(Mp / GB_BM), nt = (int)(Np / GB_BN);
      constexpr int WAVES = 8;   // 2 waves per SIMD: one wave's LDS/barrier phase hides under the other's MFMAs
      if (fuse && fuse->mode == 2)
        hipLaunchKernelGGL((k_gemm_big<OpB, PL, WAVES, 2, gemm_sched<F>()>), dim3((unsigned)(mt * nt)),
                           dim3(64 * WAVES), 0, s, (const typename OpB::T*)A, lda, aplane, (const typename OpB::T*)B,
                           ldb, bplane, (float*)C, ldc, (int)Kp, mt, nt, scale_ptr, *fuse);
      else if (fuse)
        hipLaunchKernelGGL((k_gemm_big<OpB, PL, WAVES, 1, gemm_sched<F>()>), dim3((unsigned)(mt * nt)),
                           dim3(64 * WAVES), 0, s, (const typename OpB::T*)A, lda, aplane, (const typename OpB::T*)B,
                           ldb, bplane, (float*)C, ldc, (int)Kp, mt, nt, scale_ptr, *fuse);
      else
        hipLaunchKernelGGL((k_gemm_big<OpB, PL, WAVES, 0, gemm_sched<F>()>), dim3((unsigned)(mt * nt)),
                           dim3(64 * WAVES), 0, s, (const typename OpB::T*)A, lda, aplane, (const typename OpB::T*)B,
                           ldb, bplane, (float*)C, ldc, (int)Kp, mt, nt, scale_ptr, FuseArgs{});
      return;
    }
  }
  if constexpr (F == F_FP64) {
    // (falls back to the 128 x 128 kernel when the large tiles would leave most CUs idle)
    if (!small_tiles && Mp % GD_BM == 0 && Np % GD_BN == 0 && kchunk % GD_BK == 0 && lda % 2 == 0 &&
        ldb % 2 == 0 && (Mp / GD_BM) * (Np / GD_BN) * Z >= 128) {
      const int mt = (int)(Mp / GD_BM), nt = (int)(Np / GD_BN);
      hipLaunchKernelGGL(k_gemm_f64, dim3((unsigned)(mt * nt), 1, (unsigned)Z), dim3(512), 0, s, (const double*)A,
                         lda, (const double*)B, ldb, (double*)C, ldc, czs, (int)kchunk, mt, nt, scale_ptr, smult);
      return;
    }
  }
  if constexpr (F == F_FP64) {
    // 64 x 64 tiles for the small Gram matrices (R <= 64, padded to 64), with 32 doubles of K per step
    if (Mp % 128 != 0 || Np % 128 != 0) {
      dim3 grid((unsigned)(Mp / 64), (unsigned)(Np / 64), (unsigned)Z);
      hipLaunchKernelGGL((k_gemm_tn<Op, PL, 64, 64, 32>), grid, dim3(256), 0, s, (const typename Op::T*)A, lda,
                         aplane, (const typename Op::T*)B, ldb, bplane, (typename Op::Acc*)C, ldc, czs, (int)kchunk,
                         scale_ptr, smult);
      return;
    }
  }
  constexpr long T = 128;
  dim3 grid((unsigned)(Mp / T), (unsigned)(Np / T), (unsigned)Z);
  hipLaunchKernelGGL((k_gemm_tn<Op, PL, T, T, GemmCfg<F>::BK>), grid, dim3(256), 0, s,
                     (const typename Op::T*)A, lda, aplane, (const typename Op::T*)B, ldb, bplane,
                     (typename Op::Acc*)C, ldc, czs, (int)kchunk, scale_ptr, smult);
}

// The 288 x 288 GEMM with the non-prime chain in its epilogue (3D, chi_1 = chi_2 = k_1 = k_2 = 12):
// M = H rows (a multiple of 288), ncols columns (a multiple of 288), Kp a multiple of 64 bytes.
template <int F>
void launch_gemm_f12(const void* A, long lda, long aplane, const void* B, long ldb, long bplane, long M, long ncols,
                     long Kp, const double* scale_ptr, const FuseArgs& fa, hipStream_t s) {
  if constexpr (F != F_FP64) {
    typedef typename std::conditional<F == F_FP32, OpF32v, typename OpOf<F>::type>::type OpB;
    const int mt = (int)(M / F12_T), nt = (int)(ncols / F12_T);
    hipLaunchKernelGGL((k_gemm_f12<OpB, FormInfo<F>::planes>), dim3((unsigned)(mt * nt)), dim3(64 * F12_WAVES), 0, s,
                       (const typename OpB::T*)A, lda, aplane, (const typename OpB::T*)B, ldb, bplane, (int)Kp, mt,
                       nt, scale_ptr, fa);
  }
}

// Gram matrices for direction j (1-based) into A_out[side] (n x n each, n = chi_j^2).
// With dT != null (derivative mode) also dA_out = dA/dbeta.
int enqueue_gram(hotrg_handle* h, const void* T, bool t_is_f64, const LocalDims& ld, int j, int side,
                 double* A_out, const void* dT = nullptr, double* dA_out = nullptr) {
  const int d = ld.d;
  long H = 1;
  for (int i = 0; i < d; ++i) H *= ld.chi[i];
  const long R = (long)ld.chi[j] * ld.chi[0];
  const GramGeo g = gram_geo(H, R);
  double* X = h->at<double>(h->plan.off_X);
  double* part = h->at<double>(h->plan.off_part);
  double* Gh = h->at<double>(h->plan.off_Gh);
  double* Gc = h->at<double>(h->plan.off_Gc);
  // storage legs: 0 = c, 1..d-1 = n_j, d = c', d+1.. = n'_j; strides row-major
  int dims2[2 * MAXD];
  long str[2 * MAXD];
  for (int i = 0; i < d; ++i) { dims2[i] = ld.chi[i]; dims2[d + i] = ld.chi[i]; }
  str[2 * d - 1] = 1;
  for (int i = 2 * d - 2; i >= 0; --i) str[i] = str[i + 1] * dims2[i + 1];
  const int sleg = side == 0 ? j : d + j;          // n_j or n'_j
  for (int which = 0; which < 2; ++which) {
    // which 0: hat, rows (side leg, c'); which 1: check, rows (side leg, c)
    const int rleg = which == 0 ? d : 0;
    PermSpec ps{};
    ps.nd = 2 * d;
    ps.nrow = 2;
    int k = 0;
    ps.od[k] = dims2[sleg]; ps.sstride[k++] = str[sleg];
    ps.od[k] = dims2[rleg]; ps.sstride[k++] = str[rleg];
    for (int l = 0; l < 2 * d; ++l) {
      if (l == sleg || l == rleg) continue;
      ps.od[k] = dims2[l]; ps.sstride[k++] = str[l];
    }
    ps.rows = R; ps.cols = g.C; ps.rows_p = g.Rp; ps.ldd = g.Cp;
    const bool by4 = ps.cols % 4 == 0 && ps.ldd % 4 == 0 && ps.od[ps.nd - 1] % 4 == 0 && ps.nd > ps.nrow;
    auto permute = [&](const void* src, double* dst) {
      if (t_is_f64 && by4)
        hipLaunchKernelGGL((k_permute4<double, double>), dim3(grid_for(g.Rp * g.Cp / 4)), dim3(256), 0, h->s,
                           (const double*)src, dst, ps, 1.0);
      else if (t_is_f64)
        hipLaunchKernelGGL((k_permute<double, double>), dim3(grid_for(g.Rp * g.Cp)), dim3(256), 0, h->s,
                           (const double*)src, dst, ps, 1.0);
      else if (by4)
        hipLaunchKernelGGL((k_permute4<float, double>), dim3(grid_for(g.Rp * g.Cp / 4)), dim3(256), 0, h->s,
                           (const float*)src, dst, ps, 1.0);
      else
        hipLaunchKernelGGL((k_permute<float, double>), dim3(grid_for(g.Rp * g.Cp)), dim3(256), 0, h->s,
                           (const float*)src, dst, ps, 1.0);
    };
    permute(T, X);
    launch_gemm<F_FP64>(X, g.Cp, 0, X, g.Cp, 0, part, g.Rp, g.Rp * g.Rp, g.Rp, g.Rp, g.Cp, g.Z, g.kchunk,
                        nullptr, 1.0, h->s);
    hipLaunchKernelGGL(k_reduce_zp<false>, dim3((unsigned)((R * R + 15) / 16)), dim3(256), 0, h->s, (const double*)part,
                       g.Rp * g.Rp, g.Rp, g.Z, (int)R, which == 0 ? Gh : Gc);
    if (dT) {
      // d(X X^T) = dX X^T + (dX X^T)^T
      double* Xd = h->at<double>(h->plan.off_Xd);
      permute(dT, Xd);
      launch_gemm<F_FP64>(Xd, g.Cp, 0, X, g.Cp, 0, part, g.Rp, g.Rp * g.Rp, g.Rp, g.Rp, g.Cp, g.Z, g.kchunk,
                          nullptr, 1.0, h->s);
      hipLaunchKernelGGL(k_reduce_zp<true>, dim3((unsigned)((R * R + 15) / 16)), dim3(256), 0, h->s, (const double*)part,
                         g.Rp * g.Rp, g.Rp, g.Z, (int)R,
                         which == 0 ? h->at<double>(h->plan.off_dGh) : h->at<double>(h->plan.off_dGc));
    }
  }
  const long n = (long)ld.chi[j] * ld.chi[j];
  if (n >= COMB_GEMM_N) {
    const long chis = ld.chi[j], chic = ld.chi[0];
    const CombGeo cg = comb_geo(chis, chic);
    double* Pm = h->at<double>(h->plan.off_comb);
    double* Qm = Pm + cg.Mp * cg.Kp;
    double* Sm = Qm + cg.Mp * cg.Kp;
    PermSpec pq{};                      // P[(fh, gh)][(r, e)] = G[(fh chic + r) R + gh chic + e]
    pq.nd = 4; pq.nrow = 2;
    pq.od[0] = (int)chis; pq.sstride[0] = chic * R;
    pq.od[1] = (int)chis; pq.sstride[1] = chic;
    pq.od[2] = (int)chic; pq.sstride[2] = R;
    pq.od[3] = (int)chic; pq.sstride[3] = 1;
    pq.rows = n; pq.cols = chic * chic; pq.rows_p = cg.Mp; pq.ldd = cg.Kp;
    hipLaunchKernelGGL((k_permute<double, double>), dim3(grid_for(cg.Mp * cg.Kp)), dim3(256), 0, h->s,
                       (const double*)Gh, Pm, pq, 1.0);
    hipLaunchKernelGGL((k_permute<double, double>), dim3(grid_for(cg.Mp * cg.Kp)), dim3(256), 0, h->s,
                       (const double*)Gc, Qm, pq, 1.0);
    launch_gemm<F_FP64>(Pm, cg.Kp, 0, Qm, cg.Kp, 0, Sm, cg.Mp, 0, cg.Mp, cg.Mp, cg.Kp, 1, cg.Kp, nullptr, 1.0,
                        h->s);
    PermSpec pa{};                      // A[(fc, fh)][(gc, gh)] = S[(fh, gh)][(fc, gc)]
    pa.nd = 4; pa.nrow = 2;
    pa.od[0] = (int)chis; pa.sstride[0] = chis;
    pa.od[1] = (int)chis; pa.sstride[1] = chis * cg.Mp;
    pa.od[2] = (int)chis; pa.sstride[2] = 1;
    pa.od[3] = (int)chis; pa.sstride[3] = cg.Mp;
    pa.rows = n; pa.cols = n; pa.rows_p = n; pa.ldd = n;
    hipLaunchKernelGGL((k_permute<double, double>), dim3(grid_for(n * n)), dim3(256), 0, h->s, (const double*)Sm,
                       A_out, pa, 1.0);
  } else {
    hipLaunchKernelGGL(k_gram_combine, dim3(grid_for(n * n)), dim3(256), 0, h->s, (const double*)Gh,
                       (const double*)Gc, ld.chi[j], ld.chi[0], A_out);
  }
  if (dT)
    hipLaunchKernelGGL(k_gram_combine_t, dim3(grid_for(n * n)), dim3(256), 0, h->s, (const double*)Gh,
                       (const double*)Gc, (const double*)h->at<double>(h->plan.off_dGh),
                       (const double*)h->at<double>(h->plan.off_dGc), ld.chi[j], ld.chi[0], dA_out);
  HIPCHK(h, hipGetLastError());
  return HOTRG_OK;
}

// The one-workgroup-per-(c, g) non-prime chain holds a thread per (nh1, nc1) pair and
// chi2 x chi2 x k2 <= 16 x 16 x 16 register/LDS blocks.
// Shapes of the MFMA prime chain: every bond dimension and k_j <= 16, chi_2 a multiple of 4
// (H <= 4096 and b <= 256 follow).
inline bool prime_mfma_ok(const Dims& dm) {
  return dm.chic <= 16 && dm.chi1 <= 16 && dm.chi2 <= 16 && dm.k1 <= 16 && dm.k2 <= 16 && dm.chi2 % 4 == 0 &&
         dm.chi2 >= 4 && dm.H <= 4096 && dm.b <= 256 && dm.H % 4 == 0;
}

// Prime chain on MFMA (3D, reduced forms) for the pair range [pr0, pr1); false, with nothing
// launched, when the form or the shape needs the VALU kernels.
template <int F>
bool launch_prime_mfma(hipStream_t s, const Dims& dm, const void* T, const void* U1, const void* U2, long pr0,
                       long pr1, typename Store<F>::T* Bop, long Kp, long bplane, const DevState* st) {
  if constexpr (F == F_FP64) {
    return false;
  } else {
    if (!prime_mfma_ok(dm)) return false;
    const dim3 g((unsigned)dm.H), t(256);
    const float *Tf = (const float*)T, *U1f = (const float*)U1, *U2f = (const float*)U2;
    const bool all16 = dm.chic == 16 && dm.chi1 == 16 && dm.chi2 == 16 && dm.k1 == 16 && dm.k2 == 16;
    switch (all16 ? 0 : dm.chi2 / 4) {
      case 0: hipLaunchKernelGGL((k_pstage3m<F, 4, true>), g, t, 0, s, Tf, U1f, U2f, dm, (int)pr0, (int)pr1, Bop,
                                 Kp, bplane, st); break;
      case 1: hipLaunchKernelGGL((k_pstage3m<F, 1, false>), g, t, 0, s, Tf, U1f, U2f, dm, (int)pr0, (int)pr1, Bop,
                                 Kp, bplane, st); break;
      case 2: hipLaunchKernelGGL((k_pstage3m<F, 2, false>), g, t, 0, s, Tf, U1f, U2f, dm, (int)pr0, (int)pr1, Bop,
                                 Kp, bplane, st); break;
      case 3: hipLaunchKernelGGL((k_pstage3m<F, 3, false>), g, t, 0, s, Tf, U1f, U2f, dm, (int)pr0, (int)pr1, Bop,
                                 Kp, bplane, st); break;
      default: hipLaunchKernelGGL((k_pstage3m<F, 4, false>), g, t, 0, s, Tf, U1f, U2f, dm, (int)pr0, (int)pr1, Bop,
                                  Kp, bplane, st); break;
    }
    return true;
  }
}

inline bool nstage3c_ok(const Dims& dm) {
  return dm.chi1 <= 16 && dm.chi2 <= 16 && dm.k1 <= 16 && dm.k2 <= 16;
}

// Contraction (prime chain, bottleneck, non-prime chain + rename) for form F.
template <int F>
int enqueue_contract_f(hotrg_handle* h, const void* Tv, void* Tnv, const LocalDims& ld, const int* k) {
  typedef typename std::conditional<F == F_FP64, double, float>::type MT;
  typedef typename Store<F>::T ST;
  typedef typename OpOf<F>::type::Acc AT;
  const MT* T = (const MT*)Tv;
  MT* Tn = (MT*)Tnv;
  const Dims dm = make_dims(ld, k);
  const long H = dm.H, Mp = roundup(H, TILE_M), Kp = roundup(H, TILE_K);
  long pairs_total = 1;
  for (int j = 1; j < ld.d; ++j) pairs_total *= k[j - 1];
  long cp = chunk_pairs_for(ld, k, h->form, h->opts.chunk);
  if (h->tune_chunk > 0) cp = std::min<long>(cp, h->tune_chunk);   // never above what the plan holds
  ST* Aop = h->at<ST>(h->plan.off_Aop);
  ST* Bop = h->at<ST>(h->plan.off_Bop);
  AT* Cc = h->at<AT>(h->plan.off_Cc);
  DevState* st = h->st();
  const void* U1 = F == F_FP64 ? (const void*)h->at<double>(h->plan.off_Ut)
                               : (const void*)h->at<float>(h->plan.off_Ut32);
  const size_t ut_stride = h->plan.need.Ut / 8;   // elements per direction
  const void* U2 = F == F_FP64 ? (const void*)(h->at<double>(h->plan.off_Ut) + ut_stride)
                               : (const void*)(h->at<float>(h->plan.off_Ut32) + ut_stride);
  const void* U3 = F == F_FP64 ? (const void*)(h->at<double>(h->plan.off_Ut) + 2 * ut_stride)
                               : (const void*)(h->at<float>(h->plan.off_Ut32) + 2 * ut_stride);
  typedef typename std::conditional<F == F_FP64, double, float>::type UT;
  const long aplane = Mp * Kp;
  hipEvent_t t_all = tmark(h);
  hipLaunchKernelGGL((k_make_a<MT, F>), dim3(grid_for(aplane)), dim3(256), 0, h->s, T, (int)H, Aop, Mp, Kp, Kp,
                     0L, (const DevState*)st);
  for (long pr0 = 0; pr0 < pairs_total; pr0 += cp) {
    const long pr1 = std::min(pairs_total, pr0 + cp);
    const long ncols = (pr1 - pr0) * dm.chic * dm.b;
    const long Np = roundup(ncols, TILE_N);
    const long bplane = Np * Kp;
    hipEvent_t t0 = tmark(h);
    hipLaunchKernelGGL((k_zero_pad<ST>), dim3(grid_for((Np - ncols) * Kp + ncols * (Kp - H) + 1)), dim3(256), 0,
                       h->s, Bop, ncols, Np, H, Kp, bplane, FormInfo<F>::planes, 1);
    const bool mfma_prime = ld.d == 3 && !h->scalar_prime &&
                            launch_prime_mfma<F>(h->s, dm, T, U1, U2, pr0, pr1, Bop, Kp, bplane, st);
    if (mfma_prime)
      ;                                    // launched above
    else if (ld.d == 4 && cn4_for(dm) == 8)
      hipLaunchKernelGGL((k_pstage4<MT, UT, F, 8>), dim3((unsigned)(H * dm.chic)), dim3(256), 0, h->s, T,
                         (const UT*)U1, (const UT*)U2, (const UT*)U3, dm, (int)pr0, (int)pr1, Bop, Kp, bplane,
                         (const DevState*)st);
    else if (ld.d == 4)
      hipLaunchKernelGGL((k_pstage4<MT, UT, F, 12>), dim3((unsigned)(H * dm.chic)), dim3(256), 0, h->s, T,
                         (const UT*)U1, (const UT*)U2, (const UT*)U3, dm, (int)pr0, (int)pr1, Bop, Kp, bplane,
                         (const DevState*)st);
    else if (ld.d == 3 && dm.chi2 % 8 == 0 && !h->scalar_prime)
      hipLaunchKernelGGL((k_pstage3v<MT, UT, F, 8>), dim3((unsigned)H), dim3(256), 0, h->s, T, (const UT*)U1,
                         (const UT*)U2, dm, (int)pr0, (int)pr1, Bop, Kp, bplane, (const DevState*)st);
    else if (ld.d == 3 && dm.chi2 % 4 == 0 && !h->scalar_prime)
      hipLaunchKernelGGL((k_pstage3v<MT, UT, F, 4>), dim3((unsigned)H), dim3(256), 0, h->s, T, (const UT*)U1,
                         (const UT*)U2, dm, (int)pr0, (int)pr1, Bop, Kp, bplane, (const DevState*)st);
    else if (ld.d == 3)
      hipLaunchKernelGGL((k_pstage3<MT, UT, F>), dim3((unsigned)H), dim3(256), 0, h->s, T, (const UT*)U1,
                         (const UT*)U2, dm, (int)pr0, (int)pr1, Bop, Kp, bplane, (const DevState*)st);
    else if (ld.d == 2 && !h->scalar_prime && dm.chi1 <= 32 && (long)dm.chic * dm.b <= 1024) {
      const int pbk = std::max(1, 256 / dm.chi1);
      hipLaunchKernelGGL((k_pstage2r<MT, UT, F>), dim3((unsigned)H, (unsigned)((pr1 - pr0 + pbk - 1) / pbk)),
                         dim3(256), 0, h->s, T, (const UT*)U1, dm, (int)pr0, (int)pr1, pbk, Bop, Kp, bplane,
                         (const DevState*)st);
    } else
      hipLaunchKernelGGL((k_pstage<MT, UT, F>), dim3((unsigned)(H * dm.chic)), dim3(256), 0, h->s, T,
                         (const UT*)U1, (const UT*)U2, dm, (int)pr0, (int)pr1, Bop, Kp, bplane,
                         (const DevState*)st);
    tclose(h, HOTRG_T_PRIME, t0);
    const double* sp = nullptr;
    if (FormInfo<F>::fp16) {
      // the product is scaled back by 1 / (s_A s_B), a device scalar (no host round trip)
      hipLaunchKernelGGL(k_inv_scale_fp16, dim3(1), dim3(1), 0, h->s, st, dm.b);
      sp = &st->inv_scale;
    }
    // the non-prime chain runs in the GEMM epilogue when one 256 x 256 tile is one (c, g) block
    // (chi = 16), or in the 288 x 288 kernel of 2 x 2 blocks (chi = 12, an even number of c)
    const bool fused = FormInfo<F>::fused_ok && ld.d == 3 && dm.chi1 == 16 && dm.chi2 == 16 && dm.k1 == 16 &&
                       dm.k2 == 16 && h->opts.chunk >= 0 && !h->no_fuse && !h->tune_small_tiles;
    const bool fused12 = FormInfo<F>::fused_ok && ld.d == 3 && dm.chi1 == 12 && dm.chi2 == 12 && dm.k1 == 12 &&
                         dm.k2 == 12 && H % F12_T == 0 && ncols % F12_T == 0 && Kp % 64 == 0 &&
                         h->opts.chunk >= 0 && !h->no_fuse && !h->tune_small_tiles && !h->tune_no_f12;
    // 4D chi = 8: the W3 and W2 contractions in the GEMM epilogue (a (c, g) block is 2 x 2 tiles)
    const bool fused4 = FormInfo<F>::fused_ok && ld.d == 4 && dm.chi1 == 8 && dm.chi2 == 8 && dm.chi3 == 8 &&
                        dm.k1 == 8 && dm.k2 == 8 && dm.k3 == 8 && H % GB_BM == 0 && ncols % GB_BN == 0 &&
                        Kp % 64 == 0 && h->opts.chunk >= 0 && !h->no_fuse && !h->tune_small_tiles;
    FuseArgs fa{};
    if (fused || fused12) {
      fa.U1 = (const float*)U1;
      fa.U2 = (const float*)U2;
      fa.Tn = (float*)Tn;
      fa.Hn = (long)dm.k1 * dm.k2 * dm.chic;
      fa.chic = dm.chic;
      fa.g0 = (int)(pr0 * dm.chic);
      fa.mode = 1;
    }
    if (fused4) {
      fa.U2 = (const float*)U2;
      fa.U3 = (const float*)U3;
      fa.W2 = h->at<float>(h->plan.off_W2);
      fa.gcount = (int)((pr1 - pr0) * dm.chic);
      fa.mode = 2;
    }
    hipEvent_t t1 = tmark(h);
    if (fused12)
      launch_gemm_f12<F>(Aop, Kp, aplane, Bop, Kp, bplane, H, ncols, Kp, sp, fa, h->s);
    else
      launch_gemm<F>(Aop, Kp, aplane, Bop, Kp, bplane, Cc, Np, 0, Mp, Np, Kp, 1, Kp, sp, 1.0, h->s,
                     (fused || fused4) ? &fa : nullptr, h->tune_small_tiles);
    tclose(h, HOTRG_T_BOTTLENECK, t1);
    if (h->profiling) h->acc.flops_bottleneck += 2.0 * (double)H * (double)ncols * (double)H;
    if (fused || fused12) continue;
    hipEvent_t t2 = tmark(h);
    const long ncell = (long)dm.chic * (pr1 - pr0) * dm.chic;   // (c, g) blocks
    const int g0 = (int)(pr0 * dm.chic), gcount = (int)((pr1 - pr0) * dm.chic);
    const dim3 gnc((unsigned)(dm.chic * gcount));
    if (ld.d == 4 && fused4) {
      hipLaunchKernelGGL((k_nstage4n<AT, MT, UT, 8>), gnc, dim3(256), 0, h->s, (const AT*)h->at<AT>(h->plan.off_W2),
                         (const UT*)U1, dm, g0, gcount, Tn);
    } else if (ld.d == 4) {
      AT* W2 = h->at<AT>(h->plan.off_W2);
      if (cn4_for(dm) == 8) {
        hipLaunchKernelGGL((k_nstage4w<AT, UT, 8>), gnc, dim3(256), 0, h->s, (const AT*)Cc, Np, (const UT*)U2,
                           (const UT*)U3, dm, gcount, W2);
        hipLaunchKernelGGL((k_nstage4n<AT, MT, UT, 8>), gnc, dim3(256), 0, h->s, (const AT*)W2, (const UT*)U1, dm,
                           g0, gcount, Tn);
      } else {
        hipLaunchKernelGGL((k_nstage4w<AT, UT, 12>), gnc, dim3(256), 0, h->s, (const AT*)Cc, Np, (const UT*)U2,
                           (const UT*)U3, dm, gcount, W2);
        hipLaunchKernelGGL((k_nstage4n<AT, MT, UT, 12>), gnc, dim3(256), 0, h->s, (const AT*)W2, (const UT*)U1, dm,
                           g0, gcount, Tn);
      }
    }
    else if (ld.d == 3 && nstage3c_ok(dm) && dm.chi2 == 16)
      hipLaunchKernelGGL((k_nstage3p<AT, MT, UT, 16>), gnc, dim3(256), 0, h->s, (const AT*)Cc, Np, (const UT*)U1,
                         (const UT*)U2, dm, g0, gcount, Tn);
    else if (ld.d == 3 && nstage3c_ok(dm) && dm.chi2 == 12)
      hipLaunchKernelGGL((k_nstage3p<AT, MT, UT, 12>), gnc, dim3(256), 0, h->s, (const AT*)Cc, Np, (const UT*)U1,
                         (const UT*)U2, dm, g0, gcount, Tn);
    else if (ld.d == 3 && nstage3c_ok(dm) && dm.chi2 == 8)
      hipLaunchKernelGGL((k_nstage3p<AT, MT, UT, 8>), gnc, dim3(256), 0, h->s, (const AT*)Cc, Np, (const UT*)U1,
                         (const UT*)U2, dm, g0, gcount, Tn);
    else if (ld.d == 3 && nstage3c_ok(dm))
      hipLaunchKernelGGL((k_nstage3c<AT, MT, UT>), gnc, dim3(256), 0, h->s,
                         (const AT*)Cc, Np, (const UT*)U1, (const UT*)U2, dm, g0, gcount, Tn);
    else if (ld.d == 3)
      hipLaunchKernelGGL((k_nstage3b<AT, MT, UT>), dim3((unsigned)(dm.chic * ((gcount + 7) / 8))), dim3(256), 0,
                         h->s, (const AT*)Cc, Np, (const UT*)U1, (const UT*)U2, dm, g0, gcount, Tn);
    else if (dm.chi1 <= 32 && dm.k1 <= 32)
      hipLaunchKernelGGL((k_nstage2g<AT, MT, UT>), dim3((unsigned)(dm.chic * ((gcount + NG2 - 1) / NG2))),
                         dim3(256), 0, h->s, (const AT*)Cc, Np, (const UT*)U1, dm, g0, gcount, Tn);
    else
      hipLaunchKernelGGL((k_nstage2<AT, MT, UT>), dim3((unsigned)ncell), dim3(64), 0, h->s, (const AT*)Cc, Np,
                         (const UT*)U1, dm, g0, gcount, Tn);
    tclose(h, HOTRG_T_NONPRIME, t2);
  }
  tclose(h, HOTRG_T_CONTRACT, t_all);
  if (h->profiling) {
    // algorithmic MACs of the three stages as factorised here (all chunks of this step)
    const double c = dm.chic, b = dm.b, k1 = dm.k1, k2 = dm.k2, x1 = dm.chi1, x2 = dm.chi2, Hd = (double)H;
    const double k3 = dm.k3, x3 = dm.chi3;
    double macs = Hd * Hd * (k1 * k2 * k3 * c * b);            // bottleneck: M = K = H, N = k1 k2 k3 c b
    if (ld.d == 4) {
      macs += Hd * c * b * (k1 * x1 + k1 * k2 * x2 + k1 * k2 * k3 * x3);   // prime chain, leg by leg
      macs += c * c * k1 * k2 * k3 *                                       // non-prime chain per block
              ((x1 * x2) * (x1 * x2) * x3 * x3 * k3 + x1 * x1 * k2 * k3 * x2 * x2 + k1 * k2 * k3 * x1 * x1);
    } else if (ld.d == 3) {
      macs += Hd * c * k1 * b * x1 + Hd * c * k1 * k2 * b * x2; // prime chain: n'^check_1, then n'^check_2
      macs += c * c * k1 * k2 * (x1 * x1 * k2 * x2 * x2 + x1 * x1 * k1 * k2);  // non-prime chain
    } else {
      macs += Hd * c * k1 * x1 * x1;                            // prime chain
      macs += c * c * k1 * k1 * x1 * x1;                        // non-prime chain
    }
    h->acc.flops_contract += 2.0 * macs;
  }
  HIPCHK(h, hipGetLastError());
  return HOTRG_OK;
}

// Derivative mode (FP64 / FP32 forms): the new tensor and dT^new/dbeta.  The contraction is
// multilinear in (hat copy, check copy, isometries), so
//   dC2 = P(dT; U) + P(T; dU1, U2) + P(T; U1, dU2)          (prime chain, accumulated)
//   dC  = dA C2 + A dC2 = [dA | A] . [C2 | dC2]^T            (one GEMM over 2 Kp)
//   dT^new = N(dC; U) + N(C; dU1, U2) + N(C; U1, dU2)       (non-prime chain, accumulated)
// Operand rows hold both halves: A rows [dT | T], B rows [C2 | dC2] (row length 2 Kp).
template <int F>
int enqueue_contract_grad(hotrg_handle* h, const void* Tv, void* Tnv, const void* dTv, void* dTnv,
                          const LocalDims& ld, const int* k) {
  static_assert(F == F_FP64 || F == F_FP32, "derivative mode: FP64 and FP32 forms");
  typedef typename std::conditional<F == F_FP64, double, float>::type MT;
  typedef MT UT;
  const MT* T = (const MT*)Tv;
  const MT* dT = (const MT*)dTv;
  MT* Tn = (MT*)Tnv;
  MT* dTn = (MT*)dTnv;
  const Dims dm = make_dims(ld, k);
  const long H = dm.H, Mp = roundup(H, TILE_M), Kp = roundup(H, TILE_K), L2 = 2 * Kp;
  long pairs_total = 1;
  for (int j = 1; j < ld.d; ++j) pairs_total *= k[j - 1];
  const long cp = chunk_pairs_for(ld, k, h->form, h->opts.chunk, true);
  MT* Aop = h->at<MT>(h->plan.off_Aop);
  MT* Bop = h->at<MT>(h->plan.off_Bop);
  MT* Cc = h->at<MT>(h->plan.off_Cc);
  MT* dCc = h->at<MT>(h->plan.off_dCc);
  DevState* st = h->st();
  const size_t ut_stride = h->plan.need.Ut / 8;
  const UT* U1 = F == F_FP64 ? (const UT*)h->at<double>(h->plan.off_Ut) : (const UT*)h->at<float>(h->plan.off_Ut32);
  const UT* dU1 = F == F_FP64 ? (const UT*)h->at<double>(h->plan.off_dUt)
                              : (const UT*)h->at<float>(h->plan.off_dUt32);
  const UT* U2 = U1 + ut_stride;
  const UT* dU2 = dU1 + ut_stride;
  hipEvent_t t_all = tmark(h);
  hipLaunchKernelGGL((k_make_a<MT, F>), dim3(grid_for(Mp * Kp)), dim3(256), 0, h->s, dT, (int)H, Aop, Mp, Kp, L2,
                     0L, (const DevState*)st);
  hipLaunchKernelGGL((k_make_a<MT, F>), dim3(grid_for(Mp * Kp)), dim3(256), 0, h->s, T, (int)H, Aop, Mp, Kp, L2,
                     Kp, (const DevState*)st);
  for (long pr0 = 0; pr0 < pairs_total; pr0 += cp) {
    const long pr1 = std::min(pairs_total, pr0 + cp);
    const long ncols = (pr1 - pr0) * dm.chic * dm.b;
    const long Np = roundup(ncols, TILE_N);
    const long bplane = Np * L2;
    const int ip0 = (int)pr0, ip1 = (int)pr1;
    hipEvent_t t0 = tmark(h);
    hipLaunchKernelGGL((k_zero_pad<MT>), dim3(grid_for((Np - ncols) * L2 + 2 * ncols * (Kp - H) + 1)), dim3(256), 0,
                       h->s, Bop, ncols, Np, H, Kp, bplane, 1, 2);
    if (ld.d == 3) {
      const dim3 g((unsigned)H);
      hipLaunchKernelGGL((k_pstage3<MT, UT, F, false>), g, dim3(256), 0, h->s, T, U1, U2, dm, ip0, ip1, Bop, L2,
                         bplane, (const DevState*)st);
      hipLaunchKernelGGL((k_pstage3<MT, UT, F, false>), g, dim3(256), 0, h->s, dT, U1, U2, dm, ip0, ip1, Bop + Kp,
                         L2, bplane, (const DevState*)st);
      hipLaunchKernelGGL((k_pstage3<MT, UT, F, true>), g, dim3(256), 0, h->s, T, dU1, U2, dm, ip0, ip1, Bop + Kp,
                         L2, bplane, (const DevState*)st);
      hipLaunchKernelGGL((k_pstage3<MT, UT, F, true>), g, dim3(256), 0, h->s, T, U1, dU2, dm, ip0, ip1, Bop + Kp,
                         L2, bplane, (const DevState*)st);
    } else {
      const dim3 g((unsigned)(H * dm.chic));
      hipLaunchKernelGGL((k_pstage<MT, UT, F, false>), g, dim3(256), 0, h->s, T, U1, U2, dm, ip0, ip1, Bop, L2,
                         bplane, (const DevState*)st);
      hipLaunchKernelGGL((k_pstage<MT, UT, F, false>), g, dim3(256), 0, h->s, dT, U1, U2, dm, ip0, ip1, Bop + Kp,
                         L2, bplane, (const DevState*)st);
      hipLaunchKernelGGL((k_pstage<MT, UT, F, true>), g, dim3(256), 0, h->s, T, dU1, U2, dm, ip0, ip1, Bop + Kp,
                         L2, bplane, (const DevState*)st);
    }
    tclose(h, HOTRG_T_PRIME, t0);
    hipEvent_t t1 = tmark(h);
    launch_gemm<F>(Aop + Kp, L2, 0, Bop, L2, 0, Cc, Np, 0, Mp, Np, Kp, 1, Kp, nullptr, 1.0, h->s);
    launch_gemm<F>(Aop, L2, 0, Bop, L2, 0, dCc, Np, 0, Mp, Np, L2, 1, L2, nullptr, 1.0, h->s);
    tclose(h, HOTRG_T_BOTTLENECK, t1);
    if (h->profiling) h->acc.flops_bottleneck += 3.0 * 2.0 * (double)H * (double)ncols * (double)H;
    hipEvent_t t2 = tmark(h);
    const int g0 = ip0 * dm.chic, gcount = (ip1 - ip0) * dm.chic;
    if (ld.d == 3 && nstage3c_ok(dm)) {
      const dim3 g((unsigned)(dm.chic * gcount));
      hipLaunchKernelGGL((k_nstage3c<MT, MT, UT, false>), g, dim3(256), 0, h->s, (const MT*)Cc, Np, U1, U2, dm, g0,
                         gcount, Tn);
      hipLaunchKernelGGL((k_nstage3c<MT, MT, UT, false>), g, dim3(256), 0, h->s, (const MT*)dCc, Np, U1, U2, dm,
                         g0, gcount, dTn);
      hipLaunchKernelGGL((k_nstage3c<MT, MT, UT, true>), g, dim3(256), 0, h->s, (const MT*)Cc, Np, dU1, U2, dm, g0,
                         gcount, dTn);
      hipLaunchKernelGGL((k_nstage3c<MT, MT, UT, true>), g, dim3(256), 0, h->s, (const MT*)Cc, Np, U1, dU2, dm, g0,
                         gcount, dTn);
    } else if (ld.d == 3) {
      const dim3 g((unsigned)(dm.chic * ((gcount + 7) / 8)));
      hipLaunchKernelGGL((k_nstage3b<MT, MT, UT, false>), g, dim3(256), 0, h->s, (const MT*)Cc, Np, U1, U2, dm, g0,
                         gcount, Tn);
      hipLaunchKernelGGL((k_nstage3b<MT, MT, UT, false>), g, dim3(256), 0, h->s, (const MT*)dCc, Np, U1, U2, dm,
                         g0, gcount, dTn);
      hipLaunchKernelGGL((k_nstage3b<MT, MT, UT, true>), g, dim3(256), 0, h->s, (const MT*)Cc, Np, dU1, U2, dm, g0,
                         gcount, dTn);
      hipLaunchKernelGGL((k_nstage3b<MT, MT, UT, true>), g, dim3(256), 0, h->s, (const MT*)Cc, Np, U1, dU2, dm, g0,
                         gcount, dTn);
    } else {
      const dim3 g((unsigned)((long)dm.chic * gcount));
      hipLaunchKernelGGL((k_nstage2<MT, MT, UT, false>), g, dim3(64), 0, h->s, (const MT*)Cc, Np, U1, dm, g0, gcount,
                         Tn);
      hipLaunchKernelGGL((k_nstage2<MT, MT, UT, false>), g, dim3(64), 0, h->s, (const MT*)dCc, Np, U1, dm, g0,
                         gcount, dTn);
      hipLaunchKernelGGL((k_nstage2<MT, MT, UT, true>), g, dim3(64), 0, h->s, (const MT*)Cc, Np, dU1, dm, g0, gcount,
                         dTn);
    }
    tclose(h, HOTRG_T_NONPRIME, t2);
  }
  tclose(h, HOTRG_T_CONTRACT, t_all);
  HIPCHK(h, hipGetLastError());
  return HOTRG_OK;
}

int enqueue_contract(hotrg_handle* h, const void* T, void* Tn, const LocalDims& ld, const int* k) {
  switch (h->form) {
    case HOTRG_FP64: return enqueue_contract_f<F_FP64>(h, T, Tn, ld, k);
    case HOTRG_FP32: return enqueue_contract_f<F_FP32>(h, T, Tn, ld, k);
    case HOTRG_BF16: return enqueue_contract_f<F_BF16>(h, T, Tn, ld, k);
    case HOTRG_FP16: return enqueue_contract_f<F_FP16>(h, T, Tn, ld, k);
    case HOTRG_SPLIT_BF16: return enqueue_contract_f<F_SPLIT_BF16>(h, T, Tn, ld, k);
    case HOTRG_SPLIT_FP16: return enqueue_contract_f<F_SPLIT_FP16>(h, T, Tn, ld, k);
  }
  return fail(h, HOTRG_E_ARG, "bad precision form");
}

// Eigensolver work of one step: one descriptor per Gram matrix of a truncated direction
// (slot = 2 (j - 1) + side).  Host-side only: the descriptors depend on the dims alone.
int collect_eig(hotrg_handle* h, const LocalDims& ld, EigDesc* out) {
  const size_t am = h->plan.need.Amat / 8, wn = h->plan.need.w / 8;
  int count = 0;
  for (int j = 1; j < ld.d; ++j) {
    const int n = ld.chi[j] * ld.chi[j];
    if (n <= h->chi) continue;
    const int kj = std::min(n, h->chi);
    for (int side = 0; side < 2; ++side) {
      const int slot = (j - 1) * 2 + side;
      EigDesc e;
      e.n = n;
      e.kvec = h->grad ? n : kj;   // the derivative needs the discarded eigenvectors too
      e.A = h->at<double>(h->plan.off_A) + slot * am;
      e.w = h->at<double>(h->plan.off_w) + slot * wn;
      e.V = h->at<double>(h->plan.off_Vo) + slot * am;
      e.scratch = h->at<double>(h->plan.off_Vw) + slot * 2 * am;
      e.tail = e.w + n;   // the w slot holds chi^2 + 8 values
      e.fail = &h->st()->eig_fail;
      out[count++] = e;
    }
  }
  return count;
}

// Gram matrices (and their derivatives) of every truncated direction, into the slots of
// collect_eig.
int enqueue_grams(hotrg_handle* h, const void* T, const LocalDims& ld, const void* dT) {
  const size_t am = h->plan.need.Amat / 8;
  for (int j = 1; j < ld.d; ++j) {
    const int n = ld.chi[j] * ld.chi[j];
    if (n <= h->chi) continue;
    for (int side = 0; side < 2; ++side) {
      const int slot = (j - 1) * 2 + side;
      int rc = enqueue_gram(h, T, h->form == HOTRG_FP64, ld, j, side, h->at<double>(h->plan.off_A) + slot * am, dT,
                            dT ? h->at<double>(h->plan.off_dA) + slot * am : nullptr);
      if (rc) return rc;
    }
  }
  return HOTRG_OK;
}

// Choice and truncation of U^(j) per direction (untruncated: identity), after the
// eigensolver; in derivative mode also dU^(j).
int enqueue_choose(hotrg_handle* h, const LocalDims& ld, const int* k, const void* dT) {
  const int d = ld.d;
  const size_t ut_stride = h->plan.need.Ut / 8;
  const size_t am = h->plan.need.Amat / 8, wn = h->plan.need.w / 8;
  double* Vo = h->at<double>(h->plan.off_Vo);
  double* w = h->at<double>(h->plan.off_w);
  StepRec* rec_base = h->rec(0);
  DevState* st = h->st();
  for (int j = 1; j < d; ++j) {
    const int n = ld.chi[j] * ld.chi[j];
    double* Ut = h->at<double>(h->plan.off_Ut) + (size_t)(j - 1) * ut_stride;
    float* Ut32 = h->at<float>(h->plan.off_Ut32) + (size_t)(j - 1) * ut_stride;
    const int s0 = (j - 1) * 2, s1 = s0 + 1;
    hipLaunchKernelGGL(k_choose, dim3(1), dim3(256), 0, h->s, (const double*)(w + s0 * wn),
                       (const double*)(w + s1 * wn), (const double*)(Vo + s0 * am), (const double*)(Vo + s1 * am),
                       n, k[j - 1], n <= h->chi ? 1 : 0, multiplet_tau(h->form), Ut, Ut32, rec_base,
                       (const DevState*)st, j - 1, h->opts.choice);
    if (dT) {
      double* dUt = h->at<double>(h->plan.off_dUt) + (size_t)(j - 1) * ut_stride;
      float* dUt32 = h->at<float>(h->plan.off_dUt32) + (size_t)(j - 1) * ut_stride;
      if (n <= h->chi) {
        hipLaunchKernelGGL(k_zero_f64_f32, dim3(grid_for((long)n * n)), dim3(256), 0, h->s, dUt, dUt32,
                           (long)n * n);
      } else {
        double* dAm = h->at<double>(h->plan.off_dA);
        double* scr = h->at<double>(h->plan.off_dUw);
        hipLaunchKernelGGL(k_dU, dim3(1), dim3(256), 0, h->s, (const double*)(w + s0 * wn),
                           (const double*)(w + s1 * wn), (const double*)(Vo + s0 * am),
                           (const double*)(Vo + s1 * am), (const double*)(dAm + s0 * am),
                           (const double*)(dAm + s1 * am), n, k[j - 1], (const StepRec*)rec_base,
                           (const DevState*)st, j - 1, scr, scr + am, dUt, dUt32);
      }
    }
  }
  HIPCHK(h, hipGetLastError());
  return HOTRG_OK;
}

// Rotate the storage legs so that slot 0 holds lattice axis `axis`.
int enqueue_relayout(hotrg_handle* h, int axis) {
  const int d = h->ld.d;
  int shift = 0;
  while (h->axes[shift] != axis) ++shift;
  if (shift == 0) return HOTRG_OK;
  int dims2[2 * MAXD];
  long str[2 * MAXD];
  for (int i = 0; i < d; ++i) { dims2[i] = h->ld.chi[i]; dims2[d + i] = h->ld.chi[i]; }
  str[2 * d - 1] = 1;
  for (int i = 2 * d - 2; i >= 0; --i) str[i] = str[i + 1] * dims2[i + 1];
  PermSpec ps{};
  ps.nd = 2 * d;
  ps.nrow = d;
  long H = 1;
  for (int i = 0; i < d; ++i) {
    const int src = (i + shift) % d;
    ps.od[i] = dims2[src]; ps.sstride[i] = str[src];
    ps.od[d + i] = dims2[d + src]; ps.sstride[d + i] = str[d + src];
    H *= dims2[src];
  }
  ps.rows = H; ps.cols = H; ps.rows_p = H; ps.ldd = H;
  void* T = h->at<void>(h->plan.off_T);
  void* Tn = h->at<void>(h->plan.off_Tn);
  if (h->form == HOTRG_FP64)
    hipLaunchKernelGGL((k_permute<double, double>), dim3(grid_for(H * H)), dim3(256), 0, h->s, (const double*)T,
                       (double*)Tn, ps, 1.0);
  else
    hipLaunchKernelGGL((k_permute<float, float>), dim3(grid_for(H * H)), dim3(256), 0, h->s, (const float*)T,
                       (float*)Tn, ps, 1.0);
  if (h->grad) {
    void* dT = h->at<void>(h->plan.off_dT);
    void* dTn = h->at<void>(h->plan.off_dTn);
    if (h->form == HOTRG_FP64)
      hipLaunchKernelGGL((k_permute<double, double>), dim3(grid_for(H * H)), dim3(256), 0, h->s, (const double*)dT,
                         (double*)dTn, ps, 1.0);
    else
      hipLaunchKernelGGL((k_permute<float, float>), dim3(grid_for(H * H)), dim3(256), 0, h->s, (const float*)dT,
                         (float*)dTn, ps, 1.0);
    std::swap(h->plan.off_dT, h->plan.off_dTn);
  }
  HIPCHK(h, hipGetLastError());
  std::swap(h->plan.off_T, h->plan.off_Tn);
  LocalDims nl = h->ld;
  int na[MAXD];
  for (int i = 0; i < d; ++i) { nl.chi[i] = h->ld.chi[(i + shift) % d]; na[i] = h->axes[(i + shift) % d]; }
  h->ld = nl;
  for (int i = 0; i < d; ++i) h->axes[i] = na[i];
  return HOTRG_OK;
}

// Dims of the step about to run with the current layout, and after it (renamed:
// c^bar = n_1, n^bar_j = n_{j+1}, n^bar_{d-1} = c).
struct StepPlan {
  LocalDims ld, nl;
  int k[MAXD];
  long Hn;
};

StepPlan step_plan(const hotrg_handle* h) {
  StepPlan sp{};
  sp.ld = h->ld;
  const int d = sp.ld.d;
  for (int j = 1; j < d; ++j) sp.k[j - 1] = std::min(sp.ld.chi[j] * sp.ld.chi[j], h->chi);
  sp.nl.d = d;
  for (int j = 1; j < d; ++j) sp.nl.chi[j - 1] = sp.k[j - 1];
  sp.nl.chi[d - 1] = sp.ld.chi[0];
  sp.Hn = 1;
  for (int i = 0; i < d; ++i) sp.Hn *= sp.nl.chi[i];
  return sp;
}

bool same_dims(const LocalDims& a, const LocalDims& b) {
  if (a.d != b.d) return false;
  for (int i = 0; i < a.d; ++i)
    if (a.chi[i] != b.chi[i]) return false;
  return true;
}

// First half of a step: its record and the Gram matrices.  axis_rec < 0 records the
// natural cycle (computed on the device from the step counter).
int enqueue_step_front(hotrg_handle* h, int axis_rec) {
  const LocalDims& ld = h->ld;
  hipLaunchKernelGGL(k_rec_init, dim3(1), dim3(256), 0, h->s, h->rec(0), h->st(), axis_rec, ld.d,
                     ld.chi[0], ld.chi[1], ld.d >= 3 ? ld.chi[2] : 0, ld.d >= 4 ? ld.chi[3] : 0);
  void* dT = h->grad ? h->at<void>(h->plan.off_dT) : nullptr;
  return enqueue_grams(h, h->at<void>(h->plan.off_T), ld, dT);
}

// Second half (after the eigensolver): choice and truncation, the new tensor, trace,
// lnZ/V and normalisation.  Host state is not touched (advance_host does that).
int enqueue_step_back(hotrg_handle* h, const StepPlan& sp, hipEvent_t t_dec) {
  void* T = h->at<void>(h->plan.off_T);
  void* Tn = h->at<void>(h->plan.off_Tn);
  void* dT = h->grad ? h->at<void>(h->plan.off_dT) : nullptr;
  void* dTn = h->grad ? h->at<void>(h->plan.off_dTn) : nullptr;
  int rc = enqueue_choose(h, sp.ld, sp.k, dT);
  if (rc) return rc;
  tclose(h, HOTRG_T_DECOMP, t_dec);
  if (!h->grad)
    rc = enqueue_contract(h, T, Tn, sp.ld, sp.k);
  else if (h->form == HOTRG_FP64)
    rc = enqueue_contract_grad<F_FP64>(h, T, Tn, dT, dTn, sp.ld, sp.k);
  else
    rc = enqueue_contract_grad<F_FP32>(h, T, Tn, dT, dTn, sp.ld, sp.k);
  if (rc) return rc;
  DevState* st = h->st();
  const long Hn = sp.Hn;
  const int chic = sp.ld.chi[0];
  hipEvent_t t_tr = tmark(h);
  const int norm = h->opts.norm;
  if (norm == HOTRG_NORM_MAXABS) {
    if (h->form == HOTRG_FP64)
      hipLaunchKernelGGL((k_maxabs_raw<double>), dim3(grid_reduce(Hn * Hn)), dim3(256), 0, h->s, (const double*)Tn,
                         Hn * Hn, st);
    else
      hipLaunchKernelGGL((k_maxabs_raw<float>), dim3(grid_reduce(Hn * Hn)), dim3(256), 0, h->s, (const float*)Tn,
                         Hn * Hn, st);
  }
  if (h->form == HOTRG_FP64) {
    hipLaunchKernelGGL((k_trace_lnz<double>), dim3(1), dim3(256), 0, h->s, (const double*)Tn, (int)Hn, chic, st,
                       h->rec(0), norm);
    if (h->grad)
      hipLaunchKernelGGL((k_trace_t<double>), dim3(1), dim3(256), 0, h->s, (const double*)dTn, (int)Hn, st);
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, h->s, st);
    if (h->grad)
      hipLaunchKernelGGL((k_scale_t<double>), dim3(grid_reduce(Hn * Hn)), dim3(256), 0, h->s, (double*)Tn,
                         (double*)dTn, Hn * Hn, st);
    else
      hipLaunchKernelGGL((k_scale<double>), dim3(grid_reduce(Hn * Hn)), dim3(256), 0, h->s, (double*)Tn, Hn * Hn, st);
  } else {
    hipLaunchKernelGGL((k_trace_lnz<float>), dim3(1), dim3(256), 0, h->s, (const float*)Tn, (int)Hn, chic, st,
                       h->rec(0), norm);
    if (h->grad)
      hipLaunchKernelGGL((k_trace_t<float>), dim3(1), dim3(256), 0, h->s, (const float*)dTn, (int)Hn, st);
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, h->s, st);
    if (h->grad)
      hipLaunchKernelGGL((k_scale_t<float>), dim3(grid_reduce(Hn * Hn)), dim3(256), 0, h->s, (float*)Tn, (float*)dTn,
                         Hn * Hn, st);
    else
      hipLaunchKernelGGL((k_scale<float>), dim3(grid_reduce(Hn * Hn)), dim3(256), 0, h->s, (float*)Tn, Hn * Hn, st);
  }
  tclose(h, HOTRG_T_TRACE, t_tr);
  HIPCHK(h, hipGetLastError());
  return HOTRG_OK;
}

// Host bookkeeping of a step that was enqueued (or replayed): tensor buffers swap, the
// slots rotate to the next Current axis, dims and step count advance.
void advance_host(hotrg_handle* h, const StepPlan& sp) {
  std::swap(h->plan.off_T, h->plan.off_Tn);
  if (h->grad) std::swap(h->plan.off_dT, h->plan.off_dTn);
  const int d = sp.ld.d;
  int na[MAXD];
  for (int i = 0; i < d; ++i) na[i] = h->axes[(i + 1) % d];
  for (int i = 0; i < d; ++i) h->axes[i] = na[i];
  h->ld = sp.nl;
  h->p += 1;
}

int sync_state(hotrg_handle* h, DevState* out) {
  HIPCHK(h, hipStreamSynchronize(h->s));
  HIPCHK(h, hipMemcpy(out, h->st(), sizeof(DevState), hipMemcpyDeviceToHost));
  if (out->err) {
    h->failed = true;
    if (out->eig_fail == EIG_FAIL_NONFINITE)
      return fail(h, HOTRG_E_NUMERIC, "numeric failure on the device: non-finite entry of a tridiagonal matrix");
    if (out->eig_fail == EIG_FAIL_BISECT)
      return fail(h, HOTRG_E_NUMERIC, "numeric failure on the device: eigenvalue interval still open at the "
                                      "bisection's iteration cap");
    if (out->eig_fail)
      return fail(h, HOTRG_E_NUMERIC, "numeric failure on the device: eigenpair residual above its bound");
    return fail(h, HOTRG_E_NUMERIC, "numeric failure on the device: non-positive or non-finite trace");
  }
  return HOTRG_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

static int check_model(const hotrg_model* m, int chi, int form) {
  if (!m) return HOTRG_E_ARG;
  if (m->d < 2 || m->d > 4) return HOTRG_E_ARG;
  if (m->kind == HOTRG_ISING) {
    if (m->q != 2) return HOTRG_E_ARG;
  } else if (m->kind == HOTRG_POTTS) {
    if (m->q < 2 || m->q > 8 || m->h != 0.0) return HOTRG_E_ARG;
  } else {
    return HOTRG_E_ARG;
  }
  if (!std::isfinite(m->J) || !std::isfinite(m->h)) return HOTRG_E_ARG;
  if (chi < m->q || chi > max_chi_for(m->d, form)) return HOTRG_E_ARG;
  return HOTRG_OK;
}

// The option fields every entry point checks: form, record size, chunk, normalisation, choice.
static bool opts_valid(const hotrg_opts* o) {
  return o && form_valid(o->precision) && o->max_steps >= 1 && o->chunk >= 0 && o->record_grad >= 0 &&
         o->record_grad <= 1 && (o->norm == HOTRG_NORM_TRACE || o->norm == HOTRG_NORM_MAXABS) &&
         o->choice >= HOTRG_CHOOSE_EPSILON && o->choice <= HOTRG_CHOOSE_UPRIME &&
         !(o->record_grad && o->norm != HOTRG_NORM_TRACE);
}

size_t hotrg_workspace_bytes(const hotrg_model* model, int chi, const hotrg_opts* opts) {
  if (!opts_valid(opts) || check_model(model, chi, opts->precision) != HOTRG_OK) return 0;
  if (opts->record_grad && opts->precision != HOTRG_FP64 && opts->precision != HOTRG_FP32) return 0;
  if (opts->record_grad && model->d == 4) return 0;
  return make_plan(model->d, {model->q}, chi, opts->precision, opts->chunk, opts->max_steps, opts->record_grad != 0)
      .total;
}

static int check_init_args(const hotrg_model* model, double beta, int chi, const hotrg_opts* opts) {
  if (!opts || !model) return fail(nullptr, HOTRG_E_ARG, "model or opts is NULL");
  if (check_model(model, chi, opts->precision) != HOTRG_OK)
    return fail(nullptr, HOTRG_E_ARG, "invalid model or chi");
  if (opts->record_grad && model->d == 4) return fail(nullptr, HOTRG_E_ARG, "the derivative is available for d = 2, 3");
  if (!opts_valid(opts))
    return fail(nullptr, HOTRG_E_ARG, "invalid options (form, max_steps, chunk, norm, choice; the derivative needs "
                                      "the trace normalisation)");
  if (opts->record_grad && opts->precision != HOTRG_FP64 && opts->precision != HOTRG_FP32)
    return fail(nullptr, HOTRG_E_ARG, "the derivative is available in the FP64 and FP32 forms");
  if (opts->record_grad && !(beta > 0.0))
    return fail(nullptr, HOTRG_E_ARG, "the derivative needs beta > 0");
  if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(nullptr, HOTRG_E_ARG, "beta must be finite and >= 0");
  // W must be positive semi-definite: Ising needs sinh(beta J) >= 0, Potts e^{beta J} - 1 >= 0
  if (beta * model->J < 0.0) return fail(nullptr, HOTRG_E_NOT_PSD, "bond weight matrix is not PSD (J < 0)");
  return HOTRG_OK;
}

// A handle over `workspace` with the given plan: clears its state and records, builds the
// initial tensor (asynchronous, on `stream`).  Returns null with g_static_err set on error.
static hotrg_handle* new_handle(const hotrg_model* model, double beta, int chi, const hotrg_opts* opts,
                                void* workspace, size_t ws_bytes, void* stream, const Plan& P) {
  hotrg_handle* h = new hotrg_handle();
  h->model = *model;
  h->opts = *opts;
  h->beta = beta;
  h->chi = chi;
  h->form = opts->precision;
  h->ws = (char*)workspace;
  h->ws_bytes = ws_bytes;
  h->s = (hipStream_t)stream;
  h->plan = P;
  h->grad = opts->record_grad != 0;
  h->ld.d = model->d;
  for (int i = 0; i < model->d; ++i) { h->ld.chi[i] = model->q; h->axes[i] = i; }
  hipError_t e = hipMemsetAsync(h->ws + P.off_state, 0, P.off_T - P.off_state, h->s);   // state + records
  if (e == hipSuccess) {
    if (h->form == HOTRG_FP64)
      hipLaunchKernelGGL((k_init_tensor<double>), dim3(1), dim3(256), 0, h->s, h->at<double>(P.off_T),
                         h->grad ? h->at<double>(P.off_dT) : (double*)nullptr, model->kind, model->d, model->q, beta,
                         model->J, model->h, h->st(), opts->norm);
    else
      hipLaunchKernelGGL((k_init_tensor<float>), dim3(1), dim3(256), 0, h->s, h->at<float>(P.off_T),
                         h->grad ? h->at<float>(P.off_dT) : (float*)nullptr, model->kind, model->d, model->q, beta,
                         model->J, model->h, h->st(), opts->norm);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    g_static_err = std::string("device error in hotrg_init: ") + hipGetErrorString(e);
    delete h;
    return nullptr;
  }
  return h;
}

int hotrg_init(const hotrg_model* model, double beta, int chi, const hotrg_opts* opts, void* workspace,
               size_t ws_bytes, void* stream, hotrg_handle** out) {
  if (!out) return fail(nullptr, HOTRG_E_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_init_args(model, beta, chi, opts);
  if (rc) return rc;
  if (!workspace) return fail(nullptr, HOTRG_E_ARG, "workspace is NULL");
  Plan P = make_plan(model->d, {model->q}, chi, opts->precision, opts->chunk, opts->max_steps,
                     opts->record_grad != 0);
  if (ws_bytes < P.total) return fail(nullptr, HOTRG_E_OOM, "workspace too small");
  if (((uintptr_t)workspace) % ALIGN) return fail(nullptr, HOTRG_E_ARG, "workspace must be 256-byte aligned");
  hotrg_handle* h = new_handle(model, beta, chi, opts, workspace, ws_bytes, stream, P);
  if (!h) return HOTRG_E_DEVICE;
  *out = h;
  return HOTRG_OK;
}

static int check_tensor_args(int d, const int* dims, int chi, const hotrg_opts* opts) {
  if (d < 2 || d > 4 || !dims || !opts) return fail(nullptr, HOTRG_E_ARG, "invalid d, dims or opts");
  const int maxchi = max_chi_for(d, opts->precision);
  if (chi < 1 || chi > maxchi) return fail(nullptr, HOTRG_E_ARG, "chi out of range");
  for (int i = 0; i < d; ++i)
    if (dims[i] < 1 || dims[i] > maxchi) return fail(nullptr, HOTRG_E_ARG, "tensor dimension out of range");
  if (!opts_valid(opts) || opts->record_grad != 0)
    return fail(nullptr, HOTRG_E_ARG, "invalid options (record_grad must be 0 for a supplied tensor)");
  return HOTRG_OK;
}

size_t hotrg_tensor_workspace_bytes(int d, const int* dims, int chi, const hotrg_opts* opts) {
  if (check_tensor_args(d, dims, chi, opts) != HOTRG_OK) return 0;
  return make_plan(d, std::vector<int>(dims, dims + d), chi, opts->precision, opts->chunk, opts->max_steps).total;
}

int hotrg_init_tensor(int d, const int* dims, const double* T0_dev, int chi, const hotrg_opts* opts,
                      void* workspace, size_t ws_bytes, void* stream, hotrg_handle** out) {
  if (!out) return fail(nullptr, HOTRG_E_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_tensor_args(d, dims, chi, opts);
  if (rc) return rc;
  if (!T0_dev || !workspace) return fail(nullptr, HOTRG_E_ARG, "T0 or workspace is NULL");
  const Plan P = make_plan(d, std::vector<int>(dims, dims + d), chi, opts->precision, opts->chunk, opts->max_steps);
  if (ws_bytes < P.total) return fail(nullptr, HOTRG_E_OOM, "workspace too small");
  if (((uintptr_t)workspace) % ALIGN) return fail(nullptr, HOTRG_E_ARG, "workspace must be 256-byte aligned");
  hotrg_handle* h = new hotrg_handle();
  h->model = hotrg_model{-1, d, 0, 0.0, 0.0};
  h->opts = *opts;
  h->chi = chi;
  h->form = opts->precision;
  h->ws = (char*)workspace;
  h->ws_bytes = ws_bytes;
  h->s = (hipStream_t)stream;
  h->plan = P;
  h->ld.d = d;
  long H = 1;
  for (int i = 0; i < d; ++i) { h->ld.chi[i] = dims[i]; h->axes[i] = i; H *= dims[i]; }
  // state and step records cleared by a kernel (no memset node if a caller records the stream)
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(256), 0, h->s, (int*)(h->ws + P.off_state),
                     (int)((P.off_T - P.off_state) / sizeof(int)));
  if (opts->norm == HOTRG_NORM_MAXABS)
    hipLaunchKernelGGL((k_maxabs_raw<double>), dim3(grid_reduce(H * H)), dim3(256), 0, h->s, T0_dev, H * H, h->st());
  hipLaunchKernelGGL(k_init_user_trace, dim3(1), dim3(256), 0, h->s, T0_dev, (int)H, h->st(), opts->norm);
  if (h->form == HOTRG_FP64)
    hipLaunchKernelGGL((k_init_user_scale<double>), dim3(grid_reduce(H * H)), dim3(256), 0, h->s, T0_dev,
                       h->at<double>(P.off_T), H * H, h->st());
  else
    hipLaunchKernelGGL((k_init_user_scale<float>), dim3(grid_reduce(H * H)), dim3(256), 0, h->s, T0_dev,
                       h->at<float>(P.off_T), H * H, h->st());
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    delete h;
    return fail(nullptr, HOTRG_E_DEVICE, std::string("device error in hotrg_init_tensor: ") + hipGetErrorString(e));
  }
  *out = h;
  return HOTRG_OK;
}

int hotrg_step(hotrg_handle* h, int axis) {
  if (!h) return fail(nullptr, HOTRG_E_ARG, "handle is NULL");
  if (h->failed) return fail(h, HOTRG_E_STATE, "handle is in the failed state");
  if (axis < 0 || axis >= h->ld.d) return fail(h, HOTRG_E_ARG, "axis out of range");
  if (h->p >= h->plan.max_steps) return fail(h, HOTRG_E_STATE, "max_steps reached");
  hipEvent_t t_step = tmark(h);
  int rc = enqueue_relayout(h, axis);
  if (rc) return rc;
  const StepPlan sp = step_plan(h);
  hipEvent_t t_dec = tmark(h);
  EigDesc eig[EIG_SLOTS];
  const int ne = collect_eig(h, sp.ld, eig);
  rc = enqueue_step_front(h, axis);
  if (rc) return rc;
  if (ne > 0) {
    EigBatch eb{};
    eb.count = ne;
    for (int i = 0; i < ne; ++i) {
      eb.n[i] = eig[i].n; eb.kvec[i] = eig[i].kvec; eb.A[i] = eig[i].A; eb.w[i] = eig[i].w;
      eb.V[i] = eig[i].V; eb.scratch[i] = eig[i].scratch; eb.tail[i] = eig[i].tail; eb.fail[i] = eig[i].fail;
    }
    enqueue_tri_steps(eb, h->s);
    enqueue_eig_finish(eb, h->s);
  }
  rc = enqueue_step_back(h, sp, t_dec);
  if (rc) return rc;
  tclose(h, HOTRG_T_STEP, t_step);
  advance_host(h, sp);
  return HOTRG_OK;
}

int hotrg_log_z(hotrg_handle* h, double* lnz, int* steps) {
  if (!h) return fail(nullptr, HOTRG_E_ARG, "handle is NULL");
  DevState s;
  int rc = sync_state(h, &s);
  if (rc) return rc;
  if (lnz) *lnz = s.lnz;
  if (steps) *steps = h->p;
  return HOTRG_OK;
}

int hotrg_step_info(hotrg_handle* h, int step, hotrg_step_record* out) {
  if (!h || !out) return fail(h, HOTRG_E_ARG, "NULL argument");
  if (step < 1 || step > h->p) return fail(h, HOTRG_E_ARG, "step out of range");
  DevState s;
  int rc = sync_state(h, &s);
  if (rc) return rc;
  StepRec r;
  HIPCHK(h, hipMemcpy(&r, h->rec(step - 1), sizeof(StepRec), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  out->p = r.p;
  out->axis = r.axis;
  out->trace = r.trace;
  out->lnz_per_site = r.lnz;
  out->gu_wen = r.gu_wen;
  for (int i = 0; i < MAXD; ++i) {
    out->dims_before[i] = r.dims_before[i];
    out->chi_new[i] = r.chi_new[i];
    out->eps[i] = r.eps[i];
    out->eps_p[i] = r.eps_p[i];
    out->chose_prime[i] = r.chose_prime[i];
    out->truncated[i] = r.truncated[i];
    out->kept[i] = r.kept[i];
  }
  return HOTRG_OK;
}

int hotrg_spectrum(hotrg_handle* h, int step, int dir, int side, double* outv, int cap, int* n) {
  if (!h || !n || (cap > 0 && !outv)) return fail(h, HOTRG_E_ARG, "NULL argument");
  if (step < 1 || step > h->p || dir < 1 || dir >= h->ld.d || side < 0 || side > 1)
    return fail(h, HOTRG_E_ARG, "argument out of range");
  DevState s;
  int rc = sync_state(h, &s);
  if (rc) return rc;
  StepRec r;
  HIPCHK(h, hipMemcpy(&r, h->rec(step - 1), sizeof(StepRec), hipMemcpyDeviceToHost));
  const int avail = r.nspec[dir - 1][side];
  const int m = std::min(cap, avail);
  for (int i = 0; i < m; ++i) outv[i] = r.spec[dir - 1][side][i];
  *n = m;
  return HOTRG_OK;
}

int hotrg_grad(hotrg_handle* h, double* outv) {
  if (!h || !outv) return fail(h, HOTRG_E_ARG, "NULL argument");
  if (!h->grad) return fail(h, HOTRG_E_STATE, "the handle was created without record_grad");
  DevState s;
  int rc = sync_state(h, &s);
  if (rc) return rc;
  *outv = s.dlnz;
  return HOTRG_OK;
}

int hotrg_profile(hotrg_handle* h, int enable) {
  if (!h) return fail(nullptr, HOTRG_E_ARG, "handle is NULL");
  HIPCHK(h, hipStreamSynchronize(h->s));
  for (auto& pe : h->pending) { h->free_events.push_back(pe.a); h->free_events.push_back(pe.b); }
  h->pending.clear();
  h->acc = hotrg_timing{};
  h->profiling = enable != 0;
  return HOTRG_OK;
}

int hotrg_timings(hotrg_handle* h, hotrg_timing* out) {
  if (!h || !out) return fail(h, HOTRG_E_ARG, "NULL argument");
  HIPCHK(h, hipStreamSynchronize(h->s));
  for (auto& pe : h->pending) {
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, pe.a, pe.b));
    h->acc.ms[pe.cat] += ms;
    h->acc.count[pe.cat] += 1;
    h->free_events.push_back(pe.a);
    h->free_events.push_back(pe.b);
  }
  h->pending.clear();
  *out = h->acc;
  return HOTRG_OK;
}

void hotrg_destroy(hotrg_handle* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->s);
  for (auto& pe : h->pending) { h->free_events.push_back(pe.a); h->free_events.push_back(pe.b); }
  for (hipEvent_t e : h->free_events) (void)hipEventDestroy(e);
  delete h;
}

const char* hotrg_last_error(const hotrg_handle* h) {
  if (!h) return g_static_err.c_str();
  return h->err.c_str();
}

// ---------------------------------------------------------------------------
// Kernel-level entry points
// ---------------------------------------------------------------------------

static bool debug_dims_ok(int d, const int* dims, const int* kdims, int form = HOTRG_FP32) {
  if (d < 2 || d > 4 || !dims) return false;
  // the form only limits the contraction (kdims given); the Gram matrices are FP64 in every form
  const int maxchi = max_chi_for(d, kdims ? form : HOTRG_FP32);
  for (int i = 0; i < d; ++i)
    if (dims[i] < 1 || dims[i] > maxchi) return false;
  if (kdims)
    for (int j = 0; j < d - 1; ++j)
      if (kdims[j] < 1 || kdims[j] > maxchi || kdims[j] > dims[j + 1] * dims[j + 1]) return false;
  return true;
}

static Plan debug_plan(int d, const int* dims, const int* kdims, int form) {
  LocalDims ld;
  ld.d = d;
  for (int i = 0; i < d; ++i) ld.chi[i] = dims[i];
  int chi = 1;
  for (int i = 0; i < d; ++i) chi = std::max(chi, dims[i]);
  if (kdims)
    for (int j = 0; j < d - 1; ++j) chi = std::max(chi, kdims[j]);
  Plan P{};
  P.need = need_for(ld, chi, form, 0);
  // kdims may be smaller than min(chi^2, chi): need_for used the larger value -> still enough
  P.max_steps = 1;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = roundup(o + bytes, ALIGN); return r; };
  const Need& nd = P.need;
  long H = 1;
  for (int i = 0; i < d; ++i) H *= dims[i];
  const size_t tb = std::max(nd.T, (size_t)H * H * 8);
  P.off_state = take(sizeof(DevState));
  P.off_rec = take(sizeof(StepRec) * 2);
  P.off_T = take(tb);
  P.off_Tn = take(tb);
  P.off_Aop = take(nd.Aop);
  P.off_Bop = take(nd.Bop);
  P.off_Cc = take(nd.Cc);
  P.off_X = take(nd.X);
  P.off_part = take(nd.part);
  P.off_Gh = take(nd.G);
  P.off_Gc = take(nd.G);
  P.off_comb = take(nd.comb);
  P.off_W2 = take(nd.W2);
  P.off_A = take(EIG_SLOTS * nd.Amat);
  P.off_Vw = take(EIG_SLOTS * 2 * nd.Amat);
  P.off_Vo = take(EIG_SLOTS * nd.Amat);
  P.off_w = take(EIG_SLOTS * nd.w);
  P.off_Ut = take(MAXD * nd.Ut);
  P.off_Ut32 = take(MAXD * nd.Ut / 2 + 64);
  P.total = o;
  return P;
}

size_t hotrg_debug_workspace_bytes(int d, const int* dims, const int* kdims, int precision) {
  if (!debug_dims_ok(d, dims, kdims, precision) || !form_valid(precision)) return 0;
  return debug_plan(d, dims, kdims, precision).total;
}

// Copy a double matrix into a float buffer or keep it (device).
__global__ void k_f64_to_mt_f32(const double* src, float* dst, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}
__global__ void k_mt_f32_to_f64(const float* src, double* dst, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}
__global__ void k_copy_f64(const double* src, double* dst, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void k_maxabs_f64(const double* src, long n, DevState* st) {
  __shared__ double red[256];
  double mx = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    mx = fmax(mx, fabs(src[i]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax((unsigned long long*)&st->maxabs, __double_as_longlong(red[0]));
}

int hotrg_debug_contract(int d, const int* dims, const int* kdims, int precision, const double* T_dev,
                         const double* const* U_dev, double* Tnext_dev, void* workspace, size_t ws_bytes,
                         void* stream) {
  if (!debug_dims_ok(d, dims, kdims, precision) || !kdims || !form_valid(precision) || !T_dev || !U_dev || !Tnext_dev ||
      !workspace)
    return fail(nullptr, HOTRG_E_ARG, "invalid argument");
  for (int j = 0; j < d - 1; ++j)
    if (!U_dev[j]) return fail(nullptr, HOTRG_E_ARG, "U is NULL");
  Plan P = debug_plan(d, dims, kdims, precision);
  if (ws_bytes < P.total) return fail(nullptr, HOTRG_E_OOM, "workspace too small");
  hotrg_handle hh;
  hotrg_handle* h = &hh;
  h->form = precision;
  h->ws = (char*)workspace;
  h->ws_bytes = ws_bytes;
  h->s = (hipStream_t)stream;
  h->plan = P;
  h->opts.chunk = 0;
  h->ld.d = d;
  for (int i = 0; i < d; ++i) h->ld.chi[i] = dims[i];
  long H = 1, Hn = dims[0];
  for (int i = 0; i < d; ++i) H *= dims[i];
  for (int j = 0; j < d - 1; ++j) Hn *= kdims[j];
  const long ut_stride = P.need.Ut / 8;
  {
    const hipError_t e = hipMemsetAsync(h->ws, 0, P.off_T, h->s);
    if (e != hipSuccess) return fail(nullptr, HOTRG_E_DEVICE, std::string("hotrg_debug_contract: ") + hipGetErrorString(e));
  }
  for (int j = 0; j < d - 1; ++j) {
    const long nu = (long)dims[j + 1] * dims[j + 1] * kdims[j];
    double* U = h->at<double>(P.off_Ut) + j * ut_stride;
    float* U32 = h->at<float>(P.off_Ut32) + j * ut_stride;
    hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(nu)), dim3(256), 0, h->s, U_dev[j], U, nu);
    hipLaunchKernelGGL(k_f64_to_mt_f32, dim3(grid_for(nu)), dim3(256), 0, h->s, U_dev[j], U32, nu);
  }
  void* T = h->at<void>(P.off_T);
  void* Tn = h->at<void>(P.off_Tn);
  hipLaunchKernelGGL(k_maxabs_f64, dim3(grid_reduce(H * H)), dim3(256), 0, h->s, T_dev, H * H, h->st());
  if (precision == HOTRG_FP64) {
    hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(H * H)), dim3(256), 0, h->s, T_dev, (double*)T, H * H);
  } else {
    hipLaunchKernelGGL(k_f64_to_mt_f32, dim3(grid_for(H * H)), dim3(256), 0, h->s, T_dev, (float*)T, H * H);
  }
  int rc = enqueue_contract(h, T, Tn, h->ld, kdims);
  if (rc) return fail(nullptr, rc, h->err);   // the handle is local: its message goes to the static one
  if (precision == HOTRG_FP64)
    hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(Hn * Hn)), dim3(256), 0, h->s, (const double*)Tn, Tnext_dev,
                       Hn * Hn);
  else
    hipLaunchKernelGGL(k_mt_f32_to_f64, dim3(grid_for(Hn * Hn)), dim3(256), 0, h->s, (const float*)Tn, Tnext_dev,
                       Hn * Hn);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(h->s);
  if (e != hipSuccess) return fail(nullptr, HOTRG_E_DEVICE, std::string("hotrg_debug_contract: ") + hipGetErrorString(e));
  return HOTRG_OK;
}

int hotrg_debug_gram(int d, const int* dims, int dir, int side, const double* T_dev, double* A_dev,
                     void* workspace, size_t ws_bytes, void* stream) {
  if (!debug_dims_ok(d, dims, nullptr) || dir < 1 || dir >= d || side < 0 || side > 1 || !T_dev || !A_dev ||
      !workspace)
    return fail(nullptr, HOTRG_E_ARG, "invalid argument");
  Plan P = debug_plan(d, dims, nullptr, HOTRG_FP64);
  if (ws_bytes < P.total) return fail(nullptr, HOTRG_E_OOM, "workspace too small");
  hotrg_handle hh;
  hotrg_handle* h = &hh;
  h->form = HOTRG_FP64;
  h->ws = (char*)workspace;
  h->s = (hipStream_t)stream;
  h->plan = P;
  h->ld.d = d;
  for (int i = 0; i < d; ++i) h->ld.chi[i] = dims[i];
  int rc = enqueue_gram(h, T_dev, true, h->ld, dir, side, A_dev);
  if (rc) return fail(nullptr, rc, h->err);
  const hipError_t e = hipStreamSynchronize(h->s);
  if (e != hipSuccess) return fail(nullptr, HOTRG_E_DEVICE, std::string("hotrg_debug_gram: ") + hipGetErrorString(e));
  return HOTRG_OK;
}

size_t hotrg_debug_eigh_workspace_bytes(int n, int batch) {
  if (n < 1 || n > EIG_MAXN || batch < 1 || batch > 4) return 0;
  return (size_t)batch * 2 * n * n * 8 + ALIGN;   // reflectors and vectors, then the failure flag
}


int hotrg_debug_eigh(int n, int batch, double* A_dev, double* w_dev, double* V_dev, void* workspace,
                     size_t ws_bytes, void* stream) {
  return hotrg_debug_eigh_lead(n, batch, n, A_dev, w_dev, V_dev, nullptr, workspace, ws_bytes, stream);
}

int hotrg_debug_eigh_lead(int n, int batch, int kvec, double* A_dev, double* w_dev, double* V_dev, double* tail_dev,
                          void* workspace, size_t ws_bytes, void* stream) {
  if (n < 1 || n > EIG_MAXN || batch < 1 || batch > 4 || kvec < 1 || kvec > n || !A_dev || !w_dev || !V_dev ||
      !workspace)
    return fail(nullptr, HOTRG_E_ARG, "invalid argument");
  if (ws_bytes < hotrg_debug_eigh_workspace_bytes(n, batch)) return fail(nullptr, HOTRG_E_OOM, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  int* flag = (int*)((char*)workspace + (size_t)batch * 2 * n * n * 8);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, flag, 1);
  EigBatch eb{};
  eb.count = batch;
  for (int b = 0; b < batch; ++b) {
    eb.n[b] = n;
    eb.kvec[b] = kvec;
    eb.A[b] = A_dev + (size_t)b * n * n;
    eb.w[b] = w_dev + (size_t)b * n;
    eb.V[b] = V_dev + (size_t)b * n * n;
    eb.scratch[b] = (double*)workspace + (size_t)b * 2 * n * n;
    eb.tail[b] = tail_dev ? tail_dev + b : nullptr;
    eb.fail[b] = flag;
  }
  enqueue_tri_steps(eb, s);
  enqueue_eig_finish(eb, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, HOTRG_E_DEVICE, hipGetErrorString(e));
  int failed = 0;
  e = hipMemcpyAsync(&failed, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(nullptr, HOTRG_E_DEVICE, hipGetErrorString(e));
  if (failed) return fail(nullptr, HOTRG_E_NUMERIC, "eigensolver failure (non-finite input, no convergence or a residual "
                                                    "above the bound)");
  return HOTRG_OK;
}


// ---------------------------------------------------------------------------
// Measurement: issue rate of the MFMA instruction each precision form uses.
// ---------------------------------------------------------------------------
int hotrg_probe_mfma_rate(int precision, double* tflops, void* stream) {
  if (!tflops || !form_valid(precision)) return fail(nullptr, HOTRG_E_ARG, "invalid argument");
  hipStream_t s = (hipStream_t)stream;
  const unsigned blocks = 4096, threads = 512;
  double flops_per_mma = 0.0;
  int iters = 0;
  auto launch = [&](int it) {
    switch (precision) {
      case HOTRG_FP64: hipLaunchKernelGGL(k_mfma_loop<OpF64>, dim3(blocks), dim3(threads), 0, s, it, (float*)nullptr);
        break;
      case HOTRG_FP32: hipLaunchKernelGGL(k_mfma_loop<OpF32>, dim3(blocks), dim3(threads), 0, s, it, (float*)nullptr);
        break;
      case HOTRG_BF16: case HOTRG_SPLIT_BF16:
        hipLaunchKernelGGL(k_mfma_loop<OpBF16>, dim3(blocks), dim3(threads), 0, s, it, (float*)nullptr); break;
      default: hipLaunchKernelGGL(k_mfma_loop<OpF16>, dim3(blocks), dim3(threads), 0, s, it, (float*)nullptr);
    }
  };
  switch (precision) {
    case HOTRG_FP64: flops_per_mma = 2.0 * 16 * 16 * 4; iters = 256; break;
    case HOTRG_FP32: flops_per_mma = 2.0 * 16 * 16 * 4; iters = 512; break;
    default: flops_per_mma = 2.0 * 16 * 16 * 32; iters = 1024; break;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(nullptr, HOTRG_E_DEVICE, "event creation failed");
  // the clock settles over the first launches: a warm-up, then the fastest of three timed runs
  launch(iters);
  float ms = 0.f;
  hipError_t e = hipSuccess;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    (void)hipEventRecord(e0, s);
    launch(iters);
    (void)hipEventRecord(e1, s);
    float t = 0.f;
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess && (rep == 0 || t < ms)) ms = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(nullptr, HOTRG_E_DEVICE, hipGetErrorString(e));
  const double waves = (double)blocks * threads / 64.0;
  *tflops = waves * iters * 8.0 * flops_per_mma / (ms * 1e-3) / 1e12;
  return HOTRG_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free eigensolver entry point: the same kernels as hotrg_debug_eigh, with their
// scratch (reflectors and tridiagonal eigenvectors, 2 n^2 doubles per matrix) in a static device
// array instead of a caller workspace.  Every device the library runs on holds its own copy until
// the process ends; all calls on one device share it.
// ---------------------------------------------------------------------------
static constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;   // 16 MiB
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};   // device address of `scratch`, per device
}  // namespace

size_t hotrg_eigh_noalloc_max_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

int hotrg_eigh_noalloc(int n, int batch, double* A_dev, double* w_dev, double* V_dev, int* status_dev,
                       void* stream) {
  if (n < 1 || n > EIG_MAXN || batch < 1 || batch > 4 || !A_dev || !w_dev || !V_dev || !status_dev)
    return fail(nullptr, HOTRG_E_ARG, "invalid argument");
  const size_t need = (size_t)batch * 2 * n * n * sizeof(double);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(nullptr, HOTRG_E_ARG, "batch * 2 n^2 doubles exceed the 16 MiB static scratch of hotrg_eigh_noalloc "
                                      "(use hotrg_debug_eigh with a workspace)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, HOTRG_E_DEVICE, hipGetErrorString(e));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(nullptr, HOTRG_E_DEVICE, "device index out of range");
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
      // the host-side name `scratch` is not a device address: look the array up on this device
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(nullptr, HOTRG_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_noalloc_ptr[dev] = p;
    }
    base = (double*)g_noalloc_ptr[dev];
  }
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, status_dev, 1);
  EigBatch eb{};
  eb.count = batch;
  for (int b = 0; b < batch; ++b) {
    eb.n[b] = n;
    eb.kvec[b] = n;
    eb.A[b] = A_dev + (size_t)b * n * n;
    eb.w[b] = w_dev + (size_t)b * n;
    eb.V[b] = V_dev + (size_t)b * n * n;
    eb.scratch[b] = base + (size_t)b * 2 * n * n;
    eb.fail[b] = status_dev;
  }
  enqueue_tri_steps(eb, s);
  enqueue_eig_finish(eb, s);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, HOTRG_E_DEVICE, hipGetErrorString(e));
  return HOTRG_OK;
}

// ===========================================================================
// Batched runs
// ===========================================================================

static int batch_fail(hotrg_batch* b, int code, const std::string& msg) {
  if (b) {
    b->err = msg;
    if (code == HOTRG_E_DEVICE || code == HOTRG_E_NUMERIC) b->failed = true;
  } else {
    g_static_err = msg;
  }
  return code;
}

struct BatchLayout {
  std::vector<Plan> plans;
  size_t off_tables = 0;
  int table_cap = 0, n_tables = 0;
  size_t total = 0;
};

static constexpr int BATCH_TABLES = 8;

static int batch_layout(const hotrg_instance* inst, int n, const hotrg_opts* o, BatchLayout* L) {
  if (!inst || !o || n < 1) return HOTRG_E_ARG;
  if (o->record_grad) return HOTRG_E_ARG;     // the derivative is carried by single handles
  std::vector<Need> needs((size_t)n);
  Need shared{};
  for (int i = 0; i < n; ++i) {
    const int rc = check_init_args(&inst[i].model, inst[i].beta, inst[i].chi, o);
    if (rc) return rc;
    if (inst[i].model.d == 4) return HOTRG_E_ARG;   // batches hold 2D and 3D runs
    needs[i] = plan_need(inst[i].model.d, {inst[i].model.q}, inst[i].chi, o->precision, o->chunk, false);
    need_max(shared, needs[i]);
  }
  size_t off = 0;
  Plan S{};
  place_scratch(S, off, shared, false);
  L->table_cap = n * EIG_SLOTS;
  L->n_tables = BATCH_TABLES;
  L->off_tables = take_at(off, sizeof(EigDesc) * (size_t)L->table_cap * L->n_tables);
  L->plans.clear();
  for (int i = 0; i < n; ++i) {
    Plan P = S;
    P.need = needs[i];
    P.max_steps = o->max_steps;
    P.grad = false;
    place_private(P, off, needs[i], o->max_steps, false);
    L->plans.push_back(P);
  }
  L->total = off;
  for (auto& P : L->plans) P.total = off;
  return HOTRG_OK;
}

size_t hotrg_batch_workspace_bytes(const hotrg_instance* inst, int n, const hotrg_opts* opts) {
  BatchLayout L;
  if (batch_layout(inst, n, opts, &L) != HOTRG_OK) return 0;
  return L.total;
}

int hotrg_batch_init(const hotrg_instance* inst, int n, const hotrg_opts* opts, void* workspace, size_t ws_bytes,
                     void* stream, hotrg_batch** out) {
  if (!out) return batch_fail(nullptr, HOTRG_E_ARG, "out is NULL");
  *out = nullptr;
  if (!inst || !opts || n < 1) return batch_fail(nullptr, HOTRG_E_ARG, "instances or opts missing");
  if (opts->record_grad) return batch_fail(nullptr, HOTRG_E_ARG, "record_grad is not available for batches");
  BatchLayout L;
  const int rc = batch_layout(inst, n, opts, &L);
  if (rc) return batch_fail(nullptr, rc, "invalid instance or options");
  if (!workspace) return batch_fail(nullptr, HOTRG_E_ARG, "workspace is NULL");
  if (ws_bytes < L.total) return batch_fail(nullptr, HOTRG_E_OOM, "workspace too small");
  if (((uintptr_t)workspace) % ALIGN) return batch_fail(nullptr, HOTRG_E_ARG, "workspace must be 256-byte aligned");
  hotrg_batch* b = new hotrg_batch();
  b->n = n;
  b->opts = *opts;
  b->ws = (char*)workspace;
  b->ws_bytes = ws_bytes;
  b->s = (hipStream_t)stream;
  b->off_tables = L.off_tables;
  b->table_cap = L.table_cap;
  b->n_tables = L.n_tables;
  b->use_graphs = stream != nullptr;   // the legacy default stream cannot be recorded
  for (int i = 0; i < n; ++i) {
    hotrg_handle* h = new_handle(&inst[i].model, inst[i].beta, inst[i].chi, opts, workspace, ws_bytes, stream,
                                 L.plans[i]);
    if (!h) {
      for (auto* x : b->inst) hotrg_destroy(x);
      delete b;
      return HOTRG_E_DEVICE;
    }
    b->inst.push_back(h);
  }
  *out = b;
  return HOTRG_OK;
}

static bool desc_equal(const std::vector<EigDesc>& a, const std::vector<EigDesc>& c) {
  if (a.size() != c.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (a[i].n != c[i].n || a[i].kvec != c[i].kvec || a[i].A != c[i].A || a[i].w != c[i].w || a[i].V != c[i].V ||
        a[i].scratch != c[i].scratch || a[i].tail != c[i].tail || a[i].fail != c[i].fail)
      return false;
  return true;
}

// Device table holding `descs`: found by signature, else written into a free slot (or the
// oldest one after the stream has drained, since a pending launch may still read it).
static int batch_table(hotrg_batch* b, const std::vector<EigDesc>& descs, const EigDesc** dev) {
  *dev = nullptr;
  if (descs.empty()) return HOTRG_OK;
  for (auto& t : b->tables)
    if (desc_equal(t.key, descs)) {
      *dev = b->at<EigDesc>(b->off_tables) + (size_t)t.slot * b->table_cap;
      return HOTRG_OK;
    }
  int slot;
  if ((int)b->tables.size() < b->n_tables) {
    slot = (int)b->tables.size();
  } else {
    slot = b->next_slot;
    b->next_slot = (slot + 1) % b->n_tables;
    for (size_t i = 0; i < b->tables.size(); ++i)
      if (b->tables[i].slot == slot) { b->tables.erase(b->tables.begin() + (long)i); break; }
    if (hipStreamSynchronize(b->s) != hipSuccess) return batch_fail(b, HOTRG_E_DEVICE, "stream synchronisation failed");
  }
  EigDesc* d = b->at<EigDesc>(b->off_tables) + (size_t)slot * b->table_cap;
  if (hipMemcpy(d, descs.data(), sizeof(EigDesc) * descs.size(), hipMemcpyHostToDevice) != hipSuccess)
    return batch_fail(b, HOTRG_E_DEVICE, "descriptor upload failed");
  b->tables.push_back({descs, slot});
  *dev = d;
  return HOTRG_OK;
}

// One step of every instance: records and Gram matrices of all, one eigensolver launch,
// then choice, contraction, trace and normalisation of each in turn.
// Launch shape of the eigensolver kernels for a step's descriptor table (host copy).
struct EigLaunch {
  int ndesc = 0, maxn = 0, whole = 0, bisect_blocks = 0, max_kvec = 0;
};
static EigLaunch eig_launch(const std::vector<EigDesc>& descs) {
  EigLaunch L;
  L.ndesc = (int)descs.size();
  for (const auto& e : descs) {
    L.maxn = std::max(L.maxn, e.n);
    if (eig_split(e.n, e.kvec)) {
      L.bisect_blocks = std::max(L.bisect_blocks, (eig_nev(e.n, e.kvec) + EB_EPW - 1) / EB_EPW);
      L.max_kvec = std::max(L.max_kvec, e.kvec);
    } else {
      ++L.whole;
    }
  }
  return L;
}

static int batch_enqueue(hotrg_batch* b, const std::vector<StepPlan>& sps, const EigLaunch& L, const EigDesc* table) {
  const int ndesc = L.ndesc, maxn = L.maxn;
  for (int i = 0; i < b->n; ++i) {
    const int rc = enqueue_step_front(b->inst[i], -1);
    if (rc) return batch_fail(b, rc, "instance " + std::to_string(i) + ": " + b->inst[i]->err);
  }
  if (ndesc > 0) {
    if (maxn >= TRI_MULTI_N) {
      for (int st = 0; st < tri_lds_start(maxn); ++st)
        hipLaunchKernelGGL(k_tri_step_list, dim3((unsigned)((maxn - 1 + TRI_ROWS - 1) / TRI_ROWS), (unsigned)ndesc),
                           dim3(256), 0, b->s, table, st);
      hipLaunchKernelGGL(k_tri_finish_list, dim3((unsigned)ndesc), dim3(EIG_THREADS), 0, b->s, table);
    }
    if (L.whole) hipLaunchKernelGGL(k_eigh_list, dim3((unsigned)ndesc), dim3(EIG_THREADS), 0, b->s, table);
    if (L.bisect_blocks) {
      hipLaunchKernelGGL(k_eig_bisect_list, dim3((unsigned)L.bisect_blocks, (unsigned)ndesc), dim3(EB_THREADS), 0, b->s,
                         table);
      hipLaunchKernelGGL(k_eig_invit_list, dim3((unsigned)ndesc), dim3(EI_THREADS), 0, b->s, table);
      hipLaunchKernelGGL(k_eig_backtr_list, dim3((unsigned)L.max_kvec, (unsigned)ndesc), dim3(64), 0, b->s, table);
    }
  }
  for (int i = 0; i < b->n; ++i) {
    const int rc = enqueue_step_back(b->inst[i], sps[i], nullptr);
    if (rc) return batch_fail(b, rc, "instance " + std::to_string(i) + ": " + b->inst[i]->err);
  }
  if (hipGetLastError() != hipSuccess) return batch_fail(b, HOTRG_E_DEVICE, "kernel launch failed");
  return HOTRG_OK;
}

// Autotuner: for every distinct (d, chi) among the instances, time the saturated contraction
// of one instance with each candidate (GEMM tile 256 x 256 or 128 x 128 for the 16-bit forms;
// chunks of the plan's size, 1/2 and 1/4 of it) and keep the fastest for all instances of
// that class.  The operands are whatever the buffers hold: the dense kernels' time does not
// depend on the values, and the tensor written is the one the first step overwrites.
int hotrg_batch_tune(hotrg_batch* b, int* nclasses) {
  if (!b) return batch_fail(nullptr, HOTRG_E_ARG, "batch is NULL");
  if (b->failed) return batch_fail(b, HOTRG_E_STATE, "batch is in the failed state");
  if (b->p > 0) return batch_fail(b, HOTRG_E_STATE, "tune before the first step");
  b->tuned.clear();
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return batch_fail(b, HOTRG_E_DEVICE, "event creation failed");
  int rc = HOTRG_OK;
  for (int i = 0; i < b->n && rc == HOTRG_OK; ++i) {
    hotrg_handle* h = b->inst[i];
    const int d = h->ld.d, chi = h->chi;
    bool seen = false;
    for (const auto& t : b->tuned) seen = seen || (t.d == d && t.chi == chi);
    if (seen) continue;
    LocalDims ld;
    ld.d = d;
    for (int j = 0; j < d; ++j) ld.chi[j] = chi;
    int k[MAXD];
    for (int j = 1; j < d; ++j) k[j - 1] = chi;
    const long base = chunk_pairs_for(ld, k, h->form, h->opts.chunk);
    const bool sixteen = h->form != HOTRG_FP64 && h->form != HOTRG_FP32;
    // GEMM variants by tile edge: 288 (3D chi = 12, non-prime chain fused), 256, 128 (16-bit forms)
    const bool f12 = d == 3 && chi == 12 && h->form != HOTRG_FP64;
    std::vector<int> tiles;
    if (f12) tiles.push_back(F12_T);
    if (h->form != HOTRG_FP64) tiles.push_back(GB_BM);
    if (sixteen) tiles.push_back(128);
    if (h->form == HOTRG_FP64) tiles.push_back(0);   // one GEMM path, chunks only
    hotrg_batch::Tuned best{d, chi, 0, 0, 1e300};   // tile: GEMM tile edge
    for (size_t v = 0; v < tiles.size() && rc == HOTRG_OK; ++v)
      for (int div = 1; div <= 4 && rc == HOTRG_OK; div *= 2) {
        const long cp = std::max(1L, base / div);
        if (div > 1 && cp == std::max(1L, base / (div / 2))) continue;
        h->tune_small_tiles = tiles[v] == 128 && sixteen;
        h->tune_no_f12 = tiles[v] != F12_T;
        h->tune_chunk = (int)cp;
        float ms = 0.f;
        for (int rep = 0; rep < 3 && rc == HOTRG_OK; ++rep) {   // first run warms up
          if (rep == 1 && hipEventRecord(e0, b->s) != hipSuccess) rc = HOTRG_E_DEVICE;
          if (rc == HOTRG_OK) rc = enqueue_contract(h, h->at<void>(h->plan.off_T), h->at<void>(h->plan.off_Tn), ld, k);
        }
        if (rc == HOTRG_OK && (hipEventRecord(e1, b->s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                               hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          rc = HOTRG_E_DEVICE;
        if (rc == HOTRG_OK && ms / 2 < best.ms) best = {d, chi, tiles[v], (int)cp, ms / 2.0};
      }
    if (rc != HOTRG_OK) break;
    b->tuned.push_back(best);
    for (auto* x : b->inst)
      if (x->ld.d == d && x->chi == chi) {
        x->tune_small_tiles = best.tile == 128 && sixteen;
        x->tune_no_f12 = best.tile != F12_T;
        x->tune_chunk = best.chunk;
      }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != HOTRG_OK) return batch_fail(b, rc, "autotuner: contraction run failed");
  if (nclasses) *nclasses = (int)b->tuned.size();
  return HOTRG_OK;
}

int hotrg_batch_tuning(hotrg_batch* b, int cls, int* d, int* chi, int* gemm_tile, int* chunk_pairs,
                       double* ms) {
  if (!b || cls < 0 || cls >= (int)b->tuned.size()) return batch_fail(b, HOTRG_E_ARG, "class out of range");
  const auto& t = b->tuned[cls];
  if (d) *d = t.d;
  if (chi) *chi = t.chi;
  if (gemm_tile) *gemm_tile = t.tile;
  if (chunk_pairs) *chunk_pairs = t.chunk;
  if (ms) *ms = t.ms;
  return HOTRG_OK;
}

int hotrg_batch_step(hotrg_batch* b) {
  if (!b) return batch_fail(nullptr, HOTRG_E_ARG, "batch is NULL");
  if (b->failed) return batch_fail(b, HOTRG_E_STATE, "batch is in the failed state");
  if (b->p >= b->opts.max_steps) return batch_fail(b, HOTRG_E_STATE, "max_steps reached");
  std::vector<StepPlan> sps((size_t)b->n);
  std::vector<EigDesc> descs;
  bool steady = true;
  for (int i = 0; i < b->n; ++i) {
    hotrg_handle* h = b->inst[i];
    sps[i] = step_plan(h);
    EigDesc e[EIG_SLOTS];
    const int c = collect_eig(h, h->ld, e);
    for (int k = 0; k < c; ++k) descs.push_back(e[k]);
    if (!same_dims(sps[i].ld, sps[i].nl)) steady = false;
  }
  const EigLaunch L = eig_launch(descs);
  const EigDesc* table = nullptr;
  int rc = batch_table(b, descs, &table);
  if (rc) return rc;
  const int parity = b->p & 1;
  if (steady && b->use_graphs) {
    // every instance keeps its dims from here on: the step is the same kernel sequence each
    // time (the step counter is read on the device), with the tensor buffers alternating
    if (!b->graph[parity]) {
      if (hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return batch_fail(b, HOTRG_E_DEVICE, "stream capture could not begin");
      rc = batch_enqueue(b, sps, L, table);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(b->s, &g);
      if (rc) {
        if (g) hipGraphDestroy(g);
        return rc;
      }
      if (ec != hipSuccess || !g) return batch_fail(b, HOTRG_E_DEVICE, "stream capture failed");
      const hipError_t ei = hipGraphInstantiate(&b->graph[parity], g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (ei != hipSuccess) {
        b->graph[parity] = nullptr;
        return batch_fail(b, HOTRG_E_DEVICE, "graph instantiation failed");
      }
    }
    if (hipGraphLaunch(b->graph[parity], b->s) != hipSuccess)
      return batch_fail(b, HOTRG_E_DEVICE, "graph launch failed");
    b->graph_launches += 1;
  } else {
    rc = batch_enqueue(b, sps, L, table);
    if (rc) return rc;
    b->eager_steps += 1;
  }
  for (int i = 0; i < b->n; ++i) advance_host(b->inst[i], sps[i]);
  b->p += 1;
  return HOTRG_OK;
}

int hotrg_batch_log_z(hotrg_batch* b, double* lnz, int* steps) {
  if (!b || !lnz) return batch_fail(b, HOTRG_E_ARG, "NULL argument");
  if (hipStreamSynchronize(b->s) != hipSuccess) {
    b->failed = true;
    return batch_fail(b, HOTRG_E_DEVICE, "stream synchronisation failed");
  }
  for (int i = 0; i < b->n; ++i) {
    DevState st;
    const int rc = sync_state(b->inst[i], &st);
    if (rc) return batch_fail(b, rc, "instance " + std::to_string(i) + ": " + b->inst[i]->err);
    lnz[i] = st.lnz;
  }
  if (steps) *steps = b->p;
  return HOTRG_OK;
}

int hotrg_batch_info(hotrg_batch* b, int* graph_launches, int* eager_steps) {
  if (!b) return batch_fail(nullptr, HOTRG_E_ARG, "batch is NULL");
  if (graph_launches) *graph_launches = b->graph_launches;
  if (eager_steps) *eager_steps = b->eager_steps;
  return HOTRG_OK;
}

hotrg_handle* hotrg_batch_instance(hotrg_batch* b, int i) {
  if (!b || i < 0 || i >= b->n) return nullptr;
  return b->inst[i];
}

void hotrg_batch_destroy(hotrg_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->s);   // no graph launch may still be running when its exec goes
  for (auto& g : b->graph)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto* h : b->inst) hotrg_destroy(h);
  delete b;
}

const char* hotrg_batch_last_error(const hotrg_batch* b) {
  if (!b) return g_static_err.c_str();
  return b->err.c_str();
}

}  // extern "C"

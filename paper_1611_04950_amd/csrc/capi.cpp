// C ABI of libslepian: plans, dispatch of the HIP kernels, least squares,
// coefficients, groups and plan files.  Declarations and argument contracts
// are in include/slepian.h.
#include <hip/hip_runtime.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <new>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <mutex>
#include <vector>

#include "slepian.h"
#include "common.h"
#include "corr_sum.h"
#include "kernels.h"
#include "trace.h"

using namespace slp;

namespace {

struct Fail {
  int status;
};

inline int hip_status(hipError_t e) { return e == hipErrorOutOfMemory ? SLEPIAN_ENOMEM : SLEPIAN_EHIP; }

#define HIPCHK(call)                          \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) {                   \
      (void)hipGetLastError();                \
      throw Fail{hip_status(e_)};             \
    }                                         \
  } while (0)

template <typename T>
T *dalloc(size_t n) {
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, (n ? n : 1) * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{SLEPIAN_ENOMEM};
  }
  return static_cast<T *>(p);
}

inline void dfree(void *p) {
  if (p) (void)hipFree(p);
}

// Owns a device allocation for the duration of a scope.
template <typename T>
struct DBuf {
  T *p = nullptr;
  explicit DBuf(size_t n) : p(dalloc<T>(n)) {}
  ~DBuf() { dfree(p); }
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
};

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (dev >= 0 && dev != prev) HIPCHK(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Bump allocator over a workspace; with base == nullptr it only measures.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

// Bytes of three-pass intermediates per batch slice (tuning override:
// SLEPIAN_SLICE_MIB).
size_t slice_budget() {
  static size_t v = [] {
    size_t mib = 256;
    if (const char *e = std::getenv("SLEPIAN_SLICE_MIB")) {
      const long t = std::atol(e);
      if (t >= 1 && t <= 65536) mib = (size_t)t;
    }
    return mib << 20;
  }();
  return v;
}
constexpr int kMaxLogL = 22;                          // N <= 2^21
constexpr double kSpanMinTol = 1e-6;                  // FP32 vectors: the span projection's smallest tolerance
constexpr double kResidualMargin = 1e-12;             // Tikhonov refinement: tracked vs recomputed residual
constexpr int64_t kTuneBatch = 64;                    // signals the plan tuner times with by default
constexpr size_t kCoeffsCap = (size_t)16 << 30;       // bytes of S_K kept for slepian_coeffs
constexpr int64_t kCoeffsChunk = 65535;               // signals per coefficient GEMM launch

int ilog2_ceil(int64_t v) {
  int l = 0;
  while (((int64_t)1 << l) < v) ++l;
  return l;
}

struct OpSet {
  int64_t off = 0;   // first column within the plan's U
  int64_t r = 0;
  int set = 0;       // column set: 0 projection / pinv, 1 Tikhonov (index of the plan's tiles)
  float *d32 = nullptr;
  double *d64 = nullptr;
  std::vector<double> d;
};

}  // namespace


struct slepian_plan_s {
  int device = 0;
  int64_t N = 0, K = 0, L = 0;
  double W = 0, eps = 0, alpha = 0;
  int precision = SLEPIAN_FP32;
  FftGeom g32, g64;
  cpx<float> *tw32[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  cpx<double> *tw64[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  float *chat32 = nullptr;
  double *chat64 = nullptr;
  FftTables<float> tb32;
  FftTables<double> tb64;
  int64_t win_lo = 0, win_hi = -1;
  std::vector<double> lam;  // eigenvalues over the window
  int64_t u_l0 = 0, u_r = 0;  // U's columns are Slepian vectors l = u_l0 .. u_l0 + u_r - 1
  double *U64 = nullptr;   // leading dimension N
  float *U32 = nullptr;    // leading dimension ldu (16-byte aligned columns)
  int64_t ldu = 0;
  OpSet proj, pinv, tik, tikm;
  double lam_Km1 = 0, lam_K = 0, eps_ach = 0;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  // all K Slepian vectors for slepian_coeffs, as the coefficient GEMM's
  // operand image: FP32 columns (leading dimension ldsk, N rounded up to 32,
  // zero past N) for FP32 plans, the BF16 hi/lo image otherwise
  float *SK = nullptr;
  void *SKimg = nullptr;
  int64_t ldsk = 0;
  std::mutex coeffs_mu;
  // U's rows laid out for the fused inverse column pass, per column set and
  // matrix mode (FP32, BF16 hi/lo); null where that pass does not apply
  void *ctile[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  // U's rows laid out for pass A with the correction's coefficients, per
  // column set and matrix mode; null where that pass does not apply
  void *ftile[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  // U's layouts for prepared band sets, built by the first band set of each
  // matrix mode (0: FP32 U^T; 1: BF16 hi/lo planes of U and U^T)
  void *mbu[2] = {nullptr, nullptr};
  std::mutex mbu_mu;
  // launch tuning (slepian_plan_opts.tune): 0 none, 1 timed at creation,
  // 2 taken from the tuning cache; the time of the chosen variant
  int tuned = 0;
  double tune_us = 0;
  int64_t tune_batch = 0;
  std::string tune_cache;  // the tuning cache named at creation (groups of this plan use it too)

  ~slepian_plan_s() {
    for (auto *p : tw32) dfree(p);
    for (auto *p : tw64) dfree(p);
    dfree(chat32);
    dfree(chat64);
    dfree(U64);
    dfree(U32);
    for (OpSet *o : {&proj, &pinv, &tik, &tikm}) {
      dfree(o->d32);
      dfree(o->d64);
    }
    dfree(ws);
    dfree(SK);
    dfree(SKimg);
    for (auto &t : ctile)
      for (void *p : t) dfree(p);
    for (auto &t : ftile)
      for (void *p : t) dfree(p);
    for (void *p : mbu) dfree(p);
  }
};

// A prepared band set: the band-sum kernel's spectrum in the FP32 product's
// layout and the modulation table; U, d and the FFT tables stay the plan's.
struct slepian_bands_s {
  slepian_plan_s *P = nullptr;
  int device = 0;
  BandSet bs;
  float *chat32 = nullptr;  // spectrum of the band-sum kernel's circulant embedding / L
  float *M = nullptr;       // band_table_rows(J) rows of ldm floats
  int64_t ldm = 0;
  int mode = 0;             // matrix mode of the correction (plan precision FP32: 0, else 1)
  MbU u;                    // U's layouts, owned by the plan
  ~slepian_bands_s() {
    dfree(chat32);
    dfree(M);
  }
};

struct slepian_group_s {
  std::vector<slepian_plan_t> plans;
  std::vector<int64_t> batch;
  int device = 0;
  int prec = SLEPIAN_FP32;
  // grouped path: a device table of per-plan operands and the spans of the
  // grouped launches (index and start arrays in one device buffer)
  std::vector<slp::GroupPlan> gp;
  slp::GroupPlan *gp_dev = nullptr;
  int *span_buf = nullptr;
  std::vector<int> span_host;
  struct Span {
    size_t off = 0;  // of idx in span_host; start follows idx
    int m = 0;
    int64_t blocks = 0;
  };
  // single_corr: single pass with the correction inside; single: without
  // (the matrix-core partial / sum / apply launches carry it); colinv_corr /
  // colinv: inverse column pass with / without the fused update.
  // Alternatives chosen by timing at the first call (autotuning):
  // partial[v]: 32 (2 - v) signals per wavefront; colinv_corr[l1][v]: 8 >> v
  // wavefronts per workgroup.
  // colfwd_corr: pass A with the coefficients' partials (L1 = 16, 32).
  // colinv_corr1: L1 = 32 plans of rank <= 32 (the single-step contraction).
  Span single_corr[14], single[14], partial[2], reduce, colfwd[6], colfwd_corr[6], row[2], colinv_corr[6][2],
      colinv_corr1[2], colinv[6], apply;
  int partial_var = 0, colinv_var[6] = {0, 0, 0, 0, 0, 0};
  bool tuned = false, tuned_from_cache = false;
  std::vector<int> grouped, other;  // plan indices
  void *ws = nullptr;               // grouped workspace (Z, partials, dC per plan)
  void *ws_other = nullptr;         // for the plans run one by one
  size_t ws_other_bytes = 0;
  hipStream_t cap = nullptr, cap2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_vec = -1;  // alignment class (bit 0: all x, bit 1: all y) the graph was captured for
  std::vector<const float *> lx;
  std::vector<float *> ly;
  ~slepian_group_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (cap) (void)hipStreamDestroy(cap);
    if (cap2) (void)hipStreamDestroy(cap2);
    dfree(gp_dev);
    dfree(span_buf);
    dfree(ws);
    dfree(ws_other);
  }
};

namespace {

typedef slepian_plan_s Plan;

// ---------------------------------------------------------------------------
// Workspace layouts (shared by the size query and the calls)
// ---------------------------------------------------------------------------

// The single-pass kernel with the correction inside reads U once per signal
// pair; beyond a few pairs the matrix-core kernels, which read it once per 64
// signals, win.
constexpr int64_t kFusedSingleMaxBatch = 8;

bool fused_single(const Plan *P, const OpSet &op, int prec, int64_t b) {
  return P->g32.single() && op.r <= kMaxRankSingle && prec == SLEPIAN_FP32 && b <= kFusedSingleMaxBatch;
}

struct ProjWs {
  cpx<float> *Z = nullptr;
  int64_t slice = 0;
  float *part = nullptr, *dC = nullptr;
};

// Pass A forms the chunk partials of U^T x itself when the plan holds its
// tile for this column set and matrix mode (FP32 or BF16 hi/lo) and one
// slice of the three-pass intermediate holds every pair of the batch
// (tuning override: SLEPIAN_FWD_CORR=0 keeps the separate partial kernel).
bool fwd_corr_enabled() {
  static const bool on = [] {
    const char *e = std::getenv("SLEPIAN_FWD_CORR");
    return !(e && std::atoi(e) == 0);
  }();
  return on;
}

bool fwd_corr_applies(const Plan *P, const OpSet &op, int mode, int64_t b) {
  if (!fwd_corr_enabled()) return false;
  if (op.r <= 0 || mode < 0 || mode > 1 || !P->ftile[op.set][mode]) return false;
  if (!colfwd_corr_ok(P->g32, (int)op.r)) return false;
  const int64_t pairs = (b + 1) / 2;
  if (pairs == 0 || (pairs + 15) / 16 > 65535) return false;
  return (int64_t)conv_workspace_pairs(P->g32, pairs, sizeof(cpx<float>), slice_budget()) >= pairs;
}

// Chunk partials of U^T x: the matrix-core partial kernel's chunks or pass
// A's column blocks, whichever path the call takes (the larger of the two).
int64_t corr_part_chunks(const Plan *P, const OpSet &op, int64_t b) {
  int64_t c = corr_nchunks(P->N, b, (int)op.r);
  if (colfwd_corr_ok(P->g32, (int)op.r)) c = std::max<int64_t>(c, colfwd_corr_chunks(P->g32));
  return c;
}

ProjWs carve_project(const Plan *P, const OpSet &op, int64_t b, Carver &cv, int prec = SLEPIAN_FP32) {
  ProjWs w;
  if (fused_single(P, op, prec, b)) return w;
  const int64_t pairs = (b + 1) / 2;
  w.slice = (int64_t)conv_workspace_pairs(P->g32, pairs, sizeof(cpx<float>), slice_budget());
  if (!P->g32.single()) w.Z = cv.take<cpx<float>>((size_t)w.slice * (size_t)P->L);
  if (op.r > 0) {
    const int rpad = corr_rpad((int)op.r);
    w.part = cv.take<float>((size_t)corr_part_chunks(P, op, b) * rpad * b);
    w.dC = cv.take<float>((size_t)b * rpad);
  }
  return w;
}

struct B64Ws {
  cpx<double> *Z = nullptr;
  int64_t slice = 0;
};

B64Ws carve_b64(const Plan *P, int64_t b, Carver &cv) {
  B64Ws w;
  const int64_t pairs = (b + 1) / 2;
  // FP64 slices get four times the FP32 budget: their column passes hold
  // fewer columns per compute unit and gain more from longer launches
  w.slice = (int64_t)conv_workspace_pairs(P->g64, pairs, sizeof(cpx<double>), 4 * slice_budget());
  if (!P->g64.single()) w.Z = cv.take<cpx<double>>((size_t)w.slice * (size_t)P->L);
  return w;
}

struct TikWs {
  float *x32, *rho32, *e32;
  double *y64, *By, *t, *u, *nBy, *nr;
  double *npart = nullptr;                    // column-norm partial sums
  double *part64 = nullptr, *dC64 = nullptr;  // FP64 correction of the starting point
  ProjWs pw;
  B64Ws bw;
};

TikWs carve_tik(const Plan *P, int64_t b, Carver &cv) {
  TikWs w;
  const size_t nb = (size_t)P->N * (size_t)b;
  w.x32 = cv.take<float>(nb);
  w.rho32 = cv.take<float>(nb);
  w.e32 = cv.take<float>(nb);
  w.y64 = cv.take<double>(nb);
  w.By = cv.take<double>(nb);
  w.t = cv.take<double>(nb);
  w.u = cv.take<double>(nb);
  w.nBy = cv.take<double>(b);
  w.nr = cv.take<double>(b);
  w.npart = cv.take<double>((size_t)b * kNormParts);
  if (P->tik.r > 0) {
    const int r = (int)P->tik.r;
    w.part64 = cv.take<double>(corr64_workspace_doubles(P->N, b, r) - (size_t)r * b);
    w.dC64 = cv.take<double>((size_t)r * b);
  }
  // the fast operators of the solve use the Tikhonov column set
  w.pw = carve_project(P, P->tikm.r > P->tik.r ? P->tikm : P->tik, b, cv);
  w.bw = carve_b64(P, b, cv);
  return w;
}

// The pseudoinverse: B y through the FP32 product into t, and the correction
// in FP64 (corr64) on top of it.
struct PinvWs {
  float *t = nullptr;
  ProjWs w;
  double *part = nullptr, *dC = nullptr;
};

PinvWs carve_pinv(const Plan *P, int64_t b, Carver &cv) {
  static const OpSet none;
  PinvWs p;
  p.t = cv.take<float>((size_t)P->N * b);
  p.w = carve_project(P, none, b, cv);
  const int r = (int)P->pinv.r;
  if (r > 0) {
    p.part = cv.take<double>(corr64_workspace_doubles(P->N, b, r) - (size_t)r * b);
    p.dC = cv.take<double>((size_t)r * b);
  }
  return p;
}

size_t op_workspace(const Plan *P, int op, int64_t b) {
  Carver cv(nullptr);
  switch (op) {
    case SLEPIAN_OP_PROJECT: {
      // the largest of the precision modes
      Carver c2(nullptr);
      carve_project(P, P->proj, b, cv, SLEPIAN_FP32);
      carve_project(P, P->proj, b, c2, SLEPIAN_MIXED);
      return std::max(cv.off, c2.off) + 256;
    }
    case SLEPIAN_OP_COEFFS: {
      // x's operand image and the GEMM's per-split partial tiles, for up to
      // kCoeffsChunk signals at a time
      const int64_t bc = std::min<int64_t>(b, kCoeffsChunk);
      cv.take<char>(coeffs_image_bytes(P->N, bc));
      cv.take<float>(coeffs_part_floats(P->N, P->K, bc));
      break;
    }
    case SLEPIAN_OP_LSQ: {
      Carver c1(nullptr), c2(nullptr);
      carve_pinv(P, b, c1);
      carve_tik(P, b, c2);
      return std::max(c1.off, c2.off) + 256;
    }
    case SLEPIAN_OP_MULTIBAND:  // b = bands x signals
      cv.take<float>((size_t)P->N * 2 * b);
      cv.take<float>((size_t)P->N * 2 * b);
      carve_project(P, P->proj, 2 * b, cv, P->precision);
      break;
    default:
      return 0;
  }
  return cv.off + 256;
}

// Workspace for a call: the caller's buffer or the plan's own.
void *get_ws(Plan *P, void *work, size_t work_bytes, size_t need) {
  if (work) {
    if (work_bytes < need) throw Fail{SLEPIAN_ENOMEM};
    return work;
  }
  if (P->ws_bytes < need) {
    (void)hipDeviceSynchronize();
    dfree(P->ws);
    P->ws = nullptr;
    P->ws_bytes = 0;
    P->ws = dalloc<char>(need);
    P->ws_bytes = need;
  }
  return P->ws;
}

// ---------------------------------------------------------------------------
// Operators
// ---------------------------------------------------------------------------

// y = beta B x + gamma x + U_op diag(d_op) U_op^T x.  The product is FP32; the
// correction follows `prec` (enum slepian_precision).
void run_fast_op(const Plan *P, const OpSet &op, float beta, float gamma, const float *x, int64_t ldx, float *y,
                 int64_t ldy, int64_t b, const ProjWs &w, hipStream_t st, int prec = SLEPIAN_FP32) {
  const int64_t N = P->N;
  const float *U = P->U32 + op.off * P->ldu;
  if (fused_single(P, op, prec, b)) {
    Corr<float> c;
    c.U = U;
    c.ldu = P->ldu;
    c.r = (int)op.r;
    c.d = op.d32;
    HIPCHK(conv_apply<float>(x, ldx, y, ldy, N, b, P->g32, P->tb32, beta, gamma, c, nullptr, 0, st));
    return;
  }
  const int mode = prec == SLEPIAN_MIXED ? 1 : (prec == SLEPIAN_BF16_RAW ? 2 : 0);
  // the coefficients U^T x ride on pass A where its tile exists
  const bool fwd = fwd_corr_applies(P, op, mode, b);
  if (op.r > 0 && !fwd) {
    HIPCHK(corr_partial_mfma(mode, x, ldx, N, b, U, P->ldu, (int)op.r, w.part, st));
    HIPCHK(corr_reduce_mfma(w.part, N, b, (int)op.r, op.d32, w.dC, st));
  }
  // the update U dC rides on the inverse column pass when its U tile fits in LDS
  const int umode = mode == 0 ? 0 : 1;
  const void *tile = P->ctile[op.set][umode];
  const bool fused =
      op.r > 0 && P->g32.v2 && !P->g32.single() && colinv_corr_ok(P->g32, ldy, b, (int)op.r) && tile;
  Corr<float> c;
  if (fused) {
    c.U = U;
    c.ldu = P->ldu;
    c.r = (int)op.r;
    c.d = op.d32;
    c.dC = w.dC;
    c.mode = umode;
    c.ut = tile;
  }
  if (fwd) {
    HIPCHK(colfwd_corr(x, ldx, N, b, P->g32, P->tb32, w.Z, P->ftile[op.set][mode], (int)op.r, mode, w.part, st));
    // the row pass sums the partials into dC on the side
    RowSum rs;
    rs.part = w.part;
    rs.d = op.d32;
    rs.dC = w.dC;
    rs.chunks = colfwd_corr_chunks(P->g32);
    rs.rpad = corr_rpad((int)op.r);
    rs.b = (int)b;
    rs.r = (int)op.r;
    rs.blocks = (int)corr_reduce_blocks((int)op.r, b);
    HIPCHK(conv_rows_inv(y, ldy, N, b, P->g32, P->tb32, beta, gamma, c, w.Z, &rs, st));
  } else {
    HIPCHK(conv_apply<float>(x, ldx, y, ldy, N, b, P->g32, P->tb32, beta, gamma, c, w.Z, w.slice, st));
  }
  if (op.r > 0 && !fused) HIPCHK(corr_apply_mfma(y, ldy, N, b, U, P->ldu, (int)op.r, w.dC, st));
}

void run_b64(const Plan *P, const double *x, int64_t ldx, double *y, int64_t ldy, int64_t b, const B64Ws &w,
             hipStream_t st) {
  HIPCHK(conv_apply<double>(x, ldx, y, ldy, P->N, b, P->g64, P->tb64, 1.0, 0.0, Corr<double>(), w.Z, w.slice, st));
}

// ---------------------------------------------------------------------------
// Setup
// ---------------------------------------------------------------------------

void upload_d(OpSet &o) {
  if (o.r == 0) return;
  std::vector<float> f(o.d.begin(), o.d.end());
  o.d32 = dalloc<float>(o.r);
  HIPCHK(hipMemcpy(o.d32, f.data(), o.r * sizeof(float), hipMemcpyHostToDevice));
  o.d64 = dalloc<double>(o.r);
  HIPCHK(hipMemcpy(o.d64, o.d.data(), o.r * sizeof(double), hipMemcpyHostToDevice));
}

// The fused inverse column pass's copies of U (both matrix modes, both
// column sets), for three-pass plans whose L1 it handles.
void build_corr_tiles(Plan *P, hipStream_t st) {
  const FftGeom &g = P->g32;
  for (const OpSet *o : {&P->proj, &P->tik}) {
    if (o->r <= 0 || !colfwd_corr_ok(g, (int)o->r)) continue;
    for (int mode = 0; mode < 2; ++mode) {
      if (P->ftile[o->set][mode]) continue;  // depends on the geometry only
      void *t = dalloc<char>(fwd_tile_bytes(g, (int)o->r));
      P->ftile[o->set][mode] = t;
      HIPCHK(build_fwd_tile(P->U32 + o->off * P->ldu, P->ldu, (int)P->N, (int)o->r, g, mode, t, st));
    }
  }
  if (!g.v2 || g.single() || !colinv_corr_tiled(g)) {
    HIPCHK(hipStreamSynchronize(st));
    return;
  }
  for (const OpSet *o : {&P->proj, &P->tik}) {
    if (o->r <= 0) continue;
    for (int mode = 0; mode < 2; ++mode) {
      void *t = dalloc<char>(corr_tile_bytes(g.log1, g.log2, (int)o->r, mode));
      P->ctile[o->set][mode] = t;
      HIPCHK(build_corr_tile(P->U32 + o->off * P->ldu, P->ldu, (int)P->N, (int)o->r, g.log1, g.log2, mode, t, st));
    }
  }
  HIPCHK(hipStreamSynchronize(st));
}

// FP32 tables and kernel spectrum for rows of 2^row32 points (three-pass
// plans; a single-pass plan keeps its one geometry), keeping the plan's tuned
// launch choices.  spec: the kernel spectrum in the generic FP64 layout (the
// plan's FP64 tables must exist), or null to compute it here.
void build_fp32_state(Plan *P, int row32, const cpx<double> *spec, hipStream_t st) {
  const int logL = ilog2_ceil(2 * P->N);
  const int64_t L = P->L;
  const int cic = P->g32.cic, cicmax = P->g32.cicmax;
  P->g32 = make_geom(logL, logL <= Lds<float>::logE ? Lds<float>::logE : row32, true);
  P->g32.cic = cic;
  P->g32.cicmax = cicmax;
  P->tw32[0] = dalloc<cpx<float>>((size_t)1 << P->g32.logT);
  P->tw32[1] = dalloc<cpx<float>>((size_t)1 << P->g32.s);
  P->tw32[2] = dalloc<cpx<float>>((size_t)1 << (logL - P->g32.s));
  HIPCHK(build_tables<float>(P->g32, P->tw32[0], P->tw32[1], P->tw32[2], st));
  P->tb32 = FftTables<float>();
  P->tb32.tw_sub = P->tw32[0];
  P->tb32.tw_lo = P->tw32[1];
  P->tb32.tw_hi = P->tw32[2];
  if (P->g32.v2) {
    P->tw32[3] = dalloc<cpx<float>>((size_t)P->g32.R1 * P->g32.R2 * P->g32.R3);
    P->tw32[4] = dalloc<cpx<float>>((size_t)P->g32.R2 * P->g32.R3);
    HIPCHK(build_row_tables<float>(P->g32, P->tw32[3], P->tw32[4], st));
    P->tb32.row1 = P->tw32[3];
    P->tb32.row2 = P->tw32[4];
    if (!P->g32.single()) {
      P->tw32[5] = dalloc<cpx<float>>((size_t)L);
      HIPCHK(build_col_table<float>(P->g32, P->tw32[5], st));
      P->tb32.col = P->tw32[5];
    }
  }
  const FftGeom gen64 = generic_twin(P->g64);
  std::unique_ptr<DBuf<cpx<double>>> own;
  if (!spec) {
    DBuf<double> c(L);
    own.reset(new DBuf<cpx<double>>(L));
    HIPCHK(sinc_embed(c.p, L, P->N, P->W, st));
    HIPCHK(fft_forward_real64(c.p, gen64, P->tb64, own->p, st));
    spec = own->p;
    HIPCHK(hipStreamSynchronize(st));
  }
  P->chat32 = dalloc<float>(L);
  HIPCHK(spectrum_relayout<float>(spec, gen64, P->chat32, P->g32, st));
  P->tb32.chat = P->chat32;
  HIPCHK(hipStreamSynchronize(st));
}

// Frees the FP32 tables, spectrum and fused-pass U tiles (before a rebuild).
void free_fp32_state(Plan *P) {
  for (auto *&p : P->tw32) {
    dfree(p);
    p = nullptr;
  }
  dfree(P->chat32);
  P->chat32 = nullptr;
  for (auto &t : P->ctile)
    for (void *&p : t) {
      dfree(p);
      p = nullptr;
    }
  for (auto &t : P->ftile)
    for (void *&p : t) {
      dfree(p);
      p = nullptr;
    }
}

void build_fft_state(Plan *P, hipStream_t st) {
  const int logL = ilog2_ceil(2 * P->N);
  P->L = (int64_t)1 << logL;
  int row32 = Lds<float>::logE;
  if (const char *e = std::getenv("SLEPIAN_ROW_LOG2")) {
    // tuning override of the FP32 row length of the three-pass product
    const int v = std::atoi(e);
    if (v >= 9 && v <= Lds<float>::logE) row32 = v;
  }
  P->g64 = make_geom(logL, Lds<double>::logE, true);
  const int64_t L = P->L;
  P->tw64[0] = dalloc<cpx<double>>((size_t)1 << P->g64.logT);
  P->tw64[1] = dalloc<cpx<double>>((size_t)1 << P->g64.s);
  P->tw64[2] = dalloc<cpx<double>>((size_t)1 << (logL - P->g64.s));
  HIPCHK(build_tables<double>(P->g64, P->tw64[0], P->tw64[1], P->tw64[2], st));
  P->tb64.tw_sub = P->tw64[0];
  P->tb64.tw_lo = P->tw64[1];
  P->tb64.tw_hi = P->tw64[2];
  if (P->g64.v2) {
    P->tw64[3] = dalloc<cpx<double>>((size_t)P->g64.R1 * P->g64.R2 * P->g64.R3);
    P->tw64[4] = dalloc<cpx<double>>((size_t)P->g64.R2 * P->g64.R3);
    HIPCHK(build_row_tables<double>(P->g64, P->tw64[3], P->tw64[4], st));
    P->tb64.row1 = P->tw64[3];
    P->tb64.row2 = P->tw64[4];
    if (!P->g64.single()) {
      P->tw64[5] = dalloc<cpx<double>>((size_t)L);
      HIPCHK(build_col_table<double>(P->g64, P->tw64[5], st));
      P->tb64.col = P->tw64[5];
    }
  }
  // spectrum of the circulant embedding of B's first column (Section 4.1),
  // by the generic FP64 transform, then stored in each path's layout
  const FftGeom gen64 = generic_twin(P->g64);
  DBuf<double> c(L);
  DBuf<cpx<double>> spec(L);
  HIPCHK(sinc_embed(c.p, L, P->N, P->W, st));
  HIPCHK(fft_forward_real64(c.p, gen64, P->tb64, spec.p, st));
  build_fp32_state(P, row32, spec.p, st);
  P->chat64 = dalloc<double>(L);
  HIPCHK(spectrum_relayout<double>(spec.p, gen64, P->chat64, P->g64, st));
  P->tb64.chat = P->chat64;
  HIPCHK(hipStreamSynchronize(st));
}

struct Tridiag {
  double *a = nullptr, *e2 = nullptr, *off = nullptr;
  double gl = 0, gu = 0, pivmin = 0;
  ~Tridiag() {
    dfree(a);
    dfree(e2);
    dfree(off);
  }
};

void build_tridiag(const Plan *P, Tridiag &T, hipStream_t st) {
  const int64_t N = P->N;
  T.a = dalloc<double>(N);
  T.e2 = dalloc<double>(N);
  T.off = dalloc<double>(N);
  HIPCHK(tridiag_build(T.a, T.e2, N, P->W, st));
  // off-diagonal itself (for inverse iteration), and Gershgorin bounds
  std::vector<double> off(N > 1 ? N - 1 : 1), e2(N > 1 ? N - 1 : 1);
  const double cw = std::cos(2.0 * M_PI * P->W);
  double gl = INFINITY, gu = -INFINITY, emax = 0;
  for (int64_t n = 0; n + 1 < N; ++n) {
    off[n] = 0.5 * (double)(n + 1) * (double)(N - 1 - n);
    emax = std::max(emax, off[n] * off[n]);
  }
  for (int64_t n = 0; n < N; ++n) {
    const double h = 0.5 * (double)(N - 1) - (double)n;
    const double an = h * h * cw;
    const double r = (n > 0 ? off[n - 1] : 0.0) + (n + 1 < N ? off[n] : 0.0);
    gl = std::min(gl, an - r);
    gu = std::max(gu, an + r);
  }
  T.pivmin = DBL_MIN * std::max(1.0, emax);
  const double tn = std::max(std::fabs(gl), std::fabs(gu));
  const double pad = 2.1 * tn * DBL_EPSILON * (double)N + 4.0 * T.pivmin;
  T.gl = gl - pad;
  T.gu = gu + pad;
  if (N > 1) HIPCHK(hipMemcpyAsync(T.off, off.data(), (N - 1) * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
}

// Device memory for one batch of inverse iterations: every vector of a batch
// runs its sequential sweeps in parallel with the others, so the batch should
// hold the whole window; a quarter of the free memory, at most 16 GiB.
size_t inviter_budget() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = (size_t)8 << 30;
  return std::max<size_t>((size_t)256 << 20, std::min<size_t>((size_t)16 << 30, fr / 4));
}

// Slepian vectors l = lo..hi into V (N x (hi-lo+1), FP64, column c <-> l = lo + c).
void solve_vectors(const Plan *P, const Tridiag &T, int64_t lo, int64_t hi, double *V, hipStream_t st) {
  const int64_t N = P->N;
  const int64_t nv = hi - lo + 1;
  DBuf<double> theta(nv);
  // ascending index t = N-1-l; theta[j] <-> t = (N-1-hi) + j <-> l = hi - j
  HIPCHK(tridiag_bisect(T.a, T.e2, N, T.gl, T.gu, T.pivmin, N - 1 - hi, nv, theta.p, st));
  const size_t per = inviter_scratch_bytes(N, 1);
  int64_t cv = (int64_t)(inviter_budget() / per);
  cv = std::max<int64_t>(1, std::min(cv, nv));
  DBuf<char> scratch(inviter_scratch_bytes(N, cv));
  for (int64_t j0 = 0; j0 < nv; j0 += cv) {
    const int64_t c = std::min(cv, nv - j0);
    // theta[j0 + jj] -> column nv-1-(j0+jj) = (nv - j0 - c) + (c-1-jj)
    HIPCHK(tridiag_inviter(T.a, T.off, N, theta.p + j0, c, V + (nv - j0 - c) * N, scratch.p, 3, st));
  }
  HIPCHK(hipStreamSynchronize(st));
}

double asymptotic_width(int64_t N, double e) {
  return 2.0 / (M_PI * M_PI) * std::log((double)std::max<int64_t>(N, 2)) * std::log(1.0 / e - 1.0);
}

// One plan's eigensolve in progress: the tridiagonal matrix, the index
// window [lo, hi] (grown until its edge eigenvalues leave the thresholds),
// and the window's vectors and eigenvalues once solved.
struct EigState {
  Tridiag T;
  double thr_lo = 0, thr_hi = 0;
  int64_t h = 0, lo = 0, hi = 0;
  double *V = nullptr;  // N x (hi - lo + 1)
  std::vector<double> lam;
  int attempt = 0;
  bool done = false;
  ~EigState() { dfree(V); }
};

void eig_init(const Plan *P, EigState &E, hipStream_t st) {
  const int64_t N = P->N, K = P->K;
  E.thr_lo = P->eps;
  E.thr_hi = 1.0 - P->eps;
  if (P->alpha > 0) {
    E.thr_lo = std::min(E.thr_lo, P->alpha * (1.0 + P->alpha) * P->eps);
    E.thr_hi = std::max(E.thr_hi, 1.0 - P->eps / 3.0);
  }
  build_tridiag(P, E.T, st);
  E.h = (int64_t)(2.0 * asymptotic_width(N, std::min(E.thr_lo, 1.0 - E.thr_hi)) + 30.0);
  E.lo = std::max<int64_t>(0, K - E.h);
  E.hi = std::min<int64_t>(N - 1, K + E.h);
}

// B's eigenvalues over the solved window (FP64 Rayleigh quotients, residual
// check); true when the window brackets the thresholds, else the window is
// widened and the vectors dropped for another solve.
bool eig_check(const Plan *P, EigState &E, hipStream_t st) {
  const int64_t N = P->N, K = P->K;
  const int64_t nv = E.hi - E.lo + 1;
  std::vector<double> res(nv);
  {
    Carver c0(nullptr);
    carve_b64(P, nv, c0);
    DBuf<char> ws(c0.off + 256);
    Carver cv(ws.p);
    B64Ws bw = carve_b64(P, nv, cv);
    DBuf<double> BV((size_t)N * nv), dl(nv), dr(nv);
    run_b64(P, E.V, N, BV.p, N, nv, bw, st);
    HIPCHK(rayleigh(E.V, BV.p, N, nv, dl.p, dr.p, st));
    E.lam.assign(nv, 0.0);
    HIPCHK(hipMemcpyAsync(E.lam.data(), dl.p, nv * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(res.data(), dr.p, nv * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  for (int64_t c = 0; c < nv; ++c)
    if (!std::isfinite(E.lam[c]) || !(res[c] <= 1e-7)) throw Fail{SLEPIAN_ENOCONV};
  const bool ok_lo = E.lo == 0 || E.lam[0] >= E.thr_hi;
  const bool ok_hi = E.hi == N - 1 || E.lam[nv - 1] <= E.thr_lo;
  if (ok_lo && ok_hi) return E.done = true;
  if (++E.attempt > 12) throw Fail{SLEPIAN_ENOCONV};
  E.h *= 2;
  if (!ok_lo) E.lo = std::max<int64_t>(0, K - E.h);
  if (!ok_hi) E.hi = std::min<int64_t>(N - 1, K + E.h);
  dfree(E.V);
  E.V = nullptr;
  return false;
}

void eig_finalize(Plan *P, EigState &E, hipStream_t st) {
  const int64_t N = P->N, K = P->K;
  const int64_t lo = E.lo, hi = E.hi;
  const std::vector<double> &lam = E.lam;
  const double *V = E.V;
  const int64_t nv = hi - lo + 1;
  P->win_lo = lo;
  P->win_hi = hi;
  P->lam = lam;
  // K's gap condition (Corollary 2): lambda_{K-1} > eps, lambda_K < 1 - eps
  P->lam_Km1 = lam[K - 1 - lo];
  P->lam_K = lam[K - lo];
  if (!(P->lam_Km1 > P->eps && P->lam_K < 1.0 - P->eps)) throw Fail{SLEPIAN_EGAP};
  auto range = [&](double a, double b, int64_t &c0, int64_t &c1) {
    c0 = -1;
    c1 = -1;
    for (int64_t c = 0; c < nv; ++c)
      if (lam[c] > a && lam[c] < b) {
        if (c0 < 0) c0 = c;
        c1 = c + 1;
      }
    if (c0 < 0) {
      c0 = c1 = K - lo;
      return;
    }
    for (int64_t c = c0; c < c1; ++c)
      if (!(lam[c] > a && lam[c] < b)) throw Fail{SLEPIAN_ENOCONV};  // must be contiguous
  };
  int64_t p0, p1, t0 = 0, t1 = 0;
  range(P->eps, 1.0 - P->eps, p0, p1);
  if (P->alpha > 0) range(P->alpha * (1.0 + P->alpha) * P->eps, 1.0 - P->eps / 3.0, t0, t1);
  int64_t u0 = p0, u1 = p1;
  if (P->alpha > 0 && t1 > t0) {
    if (p1 > p0) {
      u0 = std::min(p0, t0);
      u1 = std::max(p1, t1);
    } else {
      u0 = t0;
      u1 = t1;
    }
  }
  // Lemma 4's error: max(1 - lambda over I1, lambda over I4), seen at the set edges
  double ea = 0.0;
  if (p0 > 0) ea = std::max(ea, 1.0 - lam[p0 - 1]);
  if (p1 < nv) ea = std::max(ea, lam[p1]);
  P->eps_ach = ea;
  P->u_l0 = lo + u0;
  P->u_r = u1 - u0;
  P->ldu = (N + 3) / 4 * 4;
  P->U64 = dalloc<double>((size_t)N * std::max<int64_t>(P->u_r, 1));
  P->U32 = dalloc<float>((size_t)P->ldu * std::max<int64_t>(P->u_r, 1));
  if (P->u_r > 0) {
    HIPCHK(hipMemcpyAsync(P->U64, V + u0 * N, (size_t)N * P->u_r * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(cast_f64_to_f32(P->U64, N, P->U32, P->ldu, N, P->u_r, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  dfree(E.V);
  E.V = nullptr;
  // weights of the low-rank corrections (Lemmas 4, 5, 6)
  const double al = P->alpha;
  P->proj.off = P->pinv.off = p0 - u0;
  P->proj.r = P->pinv.r = p1 - p0;
  for (int64_t c = p0; c < p1; ++c) {
    const double l = lam[c];
    const bool in_i2 = lo + c < K;
    P->proj.d.push_back(in_i2 ? 1.0 - l : -l);
    P->pinv.d.push_back(in_i2 ? 1.0 / l - l : -l);
  }
  if (al > 0) {
    P->tik.off = P->tikm.off = t0 - u0;
    P->tik.r = P->tikm.r = t1 - t0;
    for (int64_t c = t0; c < t1; ++c) {
      const double l = lam[c];
      P->tik.d.push_back(l / (l * l + al) - l / (1.0 + al));
      // refinement operator: 1/(l^2+alpha) minus its interpolation
      // 1/alpha + (1/(1+alpha) - 1/alpha) l between l = 0 and l = 1
      P->tikm.d.push_back(1.0 / (l * l + al) - (1.0 / al + (1.0 / (1.0 + al) - 1.0 / al) * l));
    }
  }
  P->tik.set = P->tikm.set = 1;
  for (OpSet *o : {&P->proj, &P->pinv, &P->tik, &P->tikm}) upload_d(*o);
  build_corr_tiles(P, st);
}

void build_eigen_state(Plan *P, hipStream_t st) {
  EigState E;
  eig_init(P, E, st);
  for (;;) {
    const int64_t nv = E.hi - E.lo + 1;
    E.V = dalloc<double>((size_t)P->N * nv);
    solve_vectors(P, E.T, E.lo, E.hi, E.V, st);
    if (eig_check(P, E, st)) break;
  }
  eig_finalize(P, E, st);
}

// Many plans' eigensolves together: the windows of all unfinished plans go
// through one batched bisection / inverse iteration / normalisation
// (eig_solve_many) per batch, batches filled up to the inverse-iteration
// memory budget; each plan's arithmetic is that of build_eigen_state.
void build_eigen_states(const std::vector<Plan *> &Ps, hipStream_t st) {
  const size_t n = Ps.size();
  std::vector<std::unique_ptr<EigState>> E(n);
  for (size_t i = 0; i < n; ++i) {
    E[i].reset(new EigState());
    eig_init(Ps[i], *E[i], st);
  }
  const size_t budget = inviter_budget();
  for (;;) {
    std::vector<size_t> pend;
    for (size_t i = 0; i < n; ++i)
      if (!E[i]->done) pend.push_back(i);
    if (pend.empty()) break;
    size_t k = 0;
    while (k < pend.size()) {
      std::vector<size_t> grp;
      size_t bytes = 0;
      for (; k < pend.size(); ++k) {
        const EigState &e = *E[pend[k]];
        const size_t sb = inviter_scratch_bytes(Ps[pend[k]]->N, e.hi - e.lo + 1);
        if (!grp.empty() && bytes + sb > budget) break;
        grp.push_back(pend[k]);
        bytes += sb;
      }
      if (grp.size() == 1 && bytes > budget) {
        // one window larger than the budget: the chunked one-plan solve
        const size_t i = grp[0];
        EigState &e = *E[i];
        e.V = dalloc<double>((size_t)Ps[i]->N * (e.hi - e.lo + 1));
        solve_vectors(Ps[i], e.T, e.lo, e.hi, e.V, st);
      } else {
        std::vector<EigJob> jobs(grp.size());
        std::vector<std::unique_ptr<DBuf<double>>> th;
        std::vector<std::unique_ptr<DBuf<char>>> scr;
        for (size_t g = 0; g < grp.size(); ++g) {
          const Plan *P = Ps[grp[g]];
          EigState &e = *E[grp[g]];
          const int64_t nv = e.hi - e.lo + 1;
          e.V = dalloc<double>((size_t)P->N * nv);
          th.emplace_back(new DBuf<double>(nv));
          scr.emplace_back(new DBuf<char>(inviter_scratch_bytes(P->N, nv)));
          EigJob &J = jobs[g];
          J.a = e.T.a;
          J.e2 = e.T.e2;
          J.off = e.T.off;
          J.N = P->N;
          J.t0 = P->N - 1 - e.hi;  // ascending index of l = hi
          J.count = nv;
          J.gl = e.T.gl;
          J.gu = e.T.gu;
          J.pivmin = e.T.pivmin;
          J.theta = th.back()->p;
          J.V = e.V;
          J.scratch = scr.back()->p;
        }
        HIPCHK(eig_solve_many(jobs.data(), (int)jobs.size(), 3, st));
      }
      for (size_t i : grp) eig_check(Ps[i], *E[i], st);
    }
  }
  for (size_t i = 0; i < n; ++i) eig_finalize(Ps[i], *E[i], st);
}

int validate_domain(int64_t N, double W, double eps, const slepian_plan_opts *o) {
  if (N < 2 || N > ((int64_t)1 << (kMaxLogL - 1))) return N < 2 ? SLEPIAN_EINVAL : SLEPIAN_ENOTSUP;
  if (!(W > 0.0 && W < 0.5)) return SLEPIAN_EINVAL;
  if (!(eps > 0.0 && eps < 0.5)) return SLEPIAN_EINVAL;
  if (o) {
    if (!(o->alpha >= 0.0) || !std::isfinite(o->alpha)) return SLEPIAN_EINVAL;
    if (o->K < 0 || o->K > N - 1) return SLEPIAN_EINVAL;
    if (o->precision < SLEPIAN_FP32 || o->precision > SLEPIAN_BF16_RAW) return SLEPIAN_EINVAL;
    if (o->tune < 0 || o->tune > 2 || o->tune_batch < 0 || o->tune_batch > 32 * (int64_t)65535) return SLEPIAN_EINVAL;
  }
  return SLEPIAN_OK;
}

template <typename F>
int guarded(F &&f) {
  try {
    return f();
  } catch (const Fail &e) {
    return e.status;
  } catch (const std::bad_alloc &) {
    return SLEPIAN_ENOMEM;
  } catch (...) {
    return SLEPIAN_EINTERNAL;
  }
}

// Bands [f - W, f + W] inside [0, 1/2] (f = 0: the baseband band), centres
// at least 2W apart, 1..kMaxBands of them.
bool parse_bands(const Plan *P, int nbands, const double *freqs, BandSet &bs) {
  if (!P || nbands < 1 || nbands > kMaxBands || !freqs) return false;
  bs.J = nbands;
  for (int i = 0; i < nbands; ++i) {
    const double f = freqs[i];
    if (!(f == 0.0 || (f >= P->W && f <= 0.5 - P->W))) return false;
    for (int k = 0; k < i; ++k)
      if (std::fabs(f - freqs[k]) < 2.0 * P->W) return false;  // bands overlap
    bs.f[i] = f;
  }
  return true;
}

bool overlapping(const float *x, int64_t ldx, const float *y, int64_t ldy, int64_t N, int64_t b) {
  if (x == y || b == 0) return false;  // in place is allowed; any other overlap is not
  const char *xa = (const char *)x, *xe = (const char *)(x + (b - 1) * ldx + N);
  const char *ya = (const char *)y, *ye = (const char *)(y + (b - 1) * ldy + N);
  return xa < ye && ya < xe;
}

// U's layouts for the modulated correction in matrix mode `mode`, built on
// first use (synchronous) and kept by the plan.
MbU mb_layout(Plan *P, int mode) {
  const int r = (int)P->proj.r;
  const int64_t N = P->N, rpad = (r + 31) / 32 * 32, ldm = mb_ldm(N);
  MbU u;
  if (r == 0) return u;
  std::lock_guard<std::mutex> lock(P->mbu_mu);
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  // mode 1: Uh, Ul (blocked, BF16) then Th, Tl; mode 0: U32b (blocked) then T32
  const size_t esz = mode == 0 ? sizeof(float) : sizeof(__bf16);
  const size_t blk = al((size_t)rpad * ldm * esz), tr = al((size_t)N * rpad * esz);
  if (!P->mbu[mode]) {
    const size_t bytes = mode == 0 ? blk + tr : 2 * blk + 2 * tr;
    char *base = dalloc<char>(bytes);
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) {
      const float *U = P->U32 + P->proj.off * P->ldu;
      if (mode == 0)
        e = mb_ulayout(0, U, P->ldu, N, r, ldm, nullptr, nullptr, reinterpret_cast<float *>(base), nullptr, nullptr,
                       reinterpret_cast<float *>(base + blk), st);
      else
        e = mb_ulayout(1, U, P->ldu, N, r, ldm, reinterpret_cast<__bf16 *>(base),
                       reinterpret_cast<__bf16 *>(base + blk), nullptr, reinterpret_cast<__bf16 *>(base + 2 * blk),
                       reinterpret_cast<__bf16 *>(base + 2 * blk + tr), nullptr, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
    if (e != hipSuccess) {
      dfree(base);
      throw Fail{hip_status(e)};
    }
    P->mbu[mode] = base;
  }
  char *base = static_cast<char *>(P->mbu[mode]);
  if (mode == 0) {
    u.U32b = reinterpret_cast<const float *>(base);
    u.T32 = reinterpret_cast<const float *>(base + blk);
  } else {
    u.Uh = reinterpret_cast<const __bf16 *>(base);
    u.Ul = reinterpret_cast<const __bf16 *>(base + blk);
    u.Th = reinterpret_cast<const __bf16 *>(base + 2 * blk);
    u.Tl = reinterpret_cast<const __bf16 *>(base + 2 * blk + tr);
  }
  return u;
}

// Workspace of a prepared band-set projection of b signals: the FFT product's
// and the modulated correction's.
size_t bands_workspace(const slepian_bands_s *B, int64_t b) {
  const Plan *P = B->P;
  Carver cv(nullptr);
  const int64_t pairs = (b + 1) / 2;
  const int64_t slice = (int64_t)conv_workspace_pairs(P->g32, pairs, sizeof(cpx<float>), slice_budget());
  if (!P->g32.single()) cv.take<cpx<float>>((size_t)slice * (size_t)P->L);
  if (P->proj.r > 0) cv.take<char>(mb_workspace_bytes(mb_shape(P->N, b, (int)P->proj.r, B->bs.J), b));
  return cv.off + 256;
}

bool bad_signal_args(const Plan *P, const void *x, int64_t ldx, const void *y, int64_t ldy, int64_t b) {
  if (!P || b < 0) return true;
  if (b == 0) return false;
  if (!x || !y || ldx < P->N || ldy < P->N) return true;
  if (b > 32 * 65535) return true;
  return false;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char *slepian_status_string(int s) {
  switch (s) {
    case SLEPIAN_OK: return "success";
    case SLEPIAN_EINVAL: return "invalid argument";
    case SLEPIAN_EGAP: return "K violates lambda_{K-1} > eps and lambda_K < 1-eps";
    case SLEPIAN_ENOMEM: return "out of memory or workspace too small";
    case SLEPIAN_EHIP: return "HIP runtime error";
    case SLEPIAN_ENOCONV: return "eigensolver check or refinement did not converge";
    case SLEPIAN_ENOTSUP: return "not supported";
    case SLEPIAN_ENONFINITE: return "non-finite value";
    case SLEPIAN_EIO: return "plan file error";
    case SLEPIAN_ESCRATCH: return "needs more scratch than the allocation-free entry point holds";
    case SLEPIAN_EINTERNAL: return "internal error";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace {

// ---- launch tuning of a plan (slepian_plan_opts.tune) ----

__global__ void k_fill_signs(float *__restrict__ x, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + (uint64_t)i * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  x[i] = (z >> 63) ? 1.0f : -1.0f;
}

struct TuneChoice {
  int row = 0, cicmax = 0, cic = 0;
  double us = 0;
};

// One cache line: "slepian-tune-v1 N W eps precision batch row cicmax cic us",
// W and eps with 17 significant digits (they read back exactly).
bool tune_cache_lookup(const char *path, const Plan *P, int64_t batch, TuneChoice &c) {
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    long long n = 0, b = 0;
    double w = 0, e = 0, us = 0;
    int prec = 0, row = 0, cmx = 0, cic = 0;
    if (std::sscanf(line, "slepian-tune-v1 %lld %lf %lf %d %lld %d %d %d %lf", &n, &w, &e, &prec, &b, &row, &cmx, &cic,
                    &us) != 9)
      continue;
    if (n != P->N || w != P->W || e != P->eps || prec != P->precision || b != batch) continue;
    if (row < 9 || row > Lds<float>::logE || (cmx != 0 && cmx != 4 && cmx != 5) || cic < 0 || cic > 2) continue;
    c.row = row;
    c.cicmax = cmx;
    c.cic = cic;
    c.us = us;
    found = true;  // the last matching line wins
  }
  std::fclose(f);
  return found;
}

void tune_cache_store(const char *path, const Plan *P, int64_t batch, const TuneChoice &c) {
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "slepian-tune-v1 %lld %.17g %.17g %d %lld %d %d %d %.3f\n", (long long)P->N, P->W, P->eps,
               P->precision, (long long)batch, c.row, c.cicmax, c.cic, c.us);
  std::fclose(f);
}

void set_fp32_geometry(Plan *P, int row, int cicmax, int cic, hipStream_t st) {
  if (P->g32.log2 != row) {
    free_fp32_state(P);
    P->g32.cicmax = cicmax;
    P->g32.cic = cic;
    build_fp32_state(P, row, nullptr, st);
    build_corr_tiles(P, st);
    return;
  }
  const bool retile = colinv_corr_tiled(P->g32) != [&] {
    FftGeom g = P->g32;
    g.cicmax = cicmax;
    return colinv_corr_tiled(g);
  }();
  P->g32.cicmax = cicmax;
  P->g32.cic = cic;
  if (retile) {
    for (auto &t : P->ctile)
      for (void *&q : t) {
        dfree(q);
        q = nullptr;
      }
    build_corr_tiles(P, st);
  }
}

// Times the plan's projection (its precision, `batch` signals of +-1) for
// each launch variant: rows of 2^13 or 2^12 points (three-pass plans), the
// update fused into the inverse column pass up to L1 = 16 or 32, and that
// pass's workgroup shapes with one pair per lane; keeps the fastest.  The variants change how
// the work is split, not what is computed.  A cache file (path may be null)
// holds earlier choices per (N, W, eps, precision, batch).
void tune_plan(Plan *P, int64_t batch, const char *cache, bool groupable, hipStream_t st) {
  const int logL = ilog2_ceil(2 * P->N);
  if (logL <= Lds<float>::logE) return;  // single pass: one launch shape
  TuneChoice best;
  if (tune_cache_lookup(cache, P, batch, best)) {
    set_fp32_geometry(P, best.row, best.cicmax, best.cic, st);
    P->tuned = 2;
    P->tune_us = best.us;
    P->tune_batch = batch;
    return;
  }
  const int64_t N = P->N;
  DBuf<float> x((size_t)N * batch), y((size_t)N * batch);
  hipLaunchKernelGGL(k_fill_signs, dim3((unsigned)(((int64_t)N * batch + 255) / 256)), dim3(256), 0, st, x.p,
                     (int64_t)N * batch, 0x7e57ull);
  HIPCHK(hipGetLastError());
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    throw Fail{SLEPIAN_EHIP};
  }
  best.us = 1e30;
  try {
    std::vector<int> rows = {Lds<float>::logE};
    // groupable: only geometries the grouped launches take (L1 <= 32)
    if (logL - (Lds<float>::logE - 1) <= (groupable ? 5 : 9)) rows.push_back(Lds<float>::logE - 1);
    for (int row : rows) {
      set_fp32_geometry(P, row, 0, 0, st);
      const int log1 = P->g32.log1;
      std::vector<int> maxes = {4};
      if (log1 == 5) maxes.push_back(5);
      for (int cmx : maxes) {
        FftGeom g = P->g32;
        g.cicmax = cmx;
        const bool fused = P->proj.r > 0 && colinv_corr_ok(g, N, batch, (int)P->proj.r);
        // one pair per lane only: groups run the fused pass that way, and with
        // the same lanes per pair a grouped call reproduces this plan's own
        // calls bit for bit (the wavefront count does not change the arithmetic)
        const std::vector<int> shapes = fused ? std::vector<int>{1, 2} : std::vector<int>{0};
        for (int cic : shapes) {
          set_fp32_geometry(P, row, cmx, cic, st);
          Carver c0(nullptr);
          carve_project(P, P->proj, batch, c0, P->precision);
          DBuf<char> ws(c0.off + 256);
          Carver cv(ws.p);
          const ProjWs w = carve_project(P, P->proj, batch, cv, P->precision);
          run_fast_op(P, P->proj, 1.0f, 0.0f, x.p, N, y.p, N, batch, w, st, P->precision);
          float t = 1e30f;
          for (int rep = 0; rep < 3; ++rep) {
            HIPCHK(hipEventRecord(e0, st));
            run_fast_op(P, P->proj, 1.0f, 0.0f, x.p, N, y.p, N, batch, w, st, P->precision);
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            t = std::min(t, ms);
          }
          if (1e3 * t < best.us) {
            best.row = row;
            best.cicmax = cmx;
            best.cic = cic;
            best.us = 1e3 * t;
          }
        }
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  set_fp32_geometry(P, best.row, best.cicmax, best.cic, st);
  P->tuned = 1;
  P->tune_us = best.us;
  P->tune_batch = batch;
  tune_cache_store(cache, P, batch, best);
}

}  // namespace

extern "C" {

int slepian_plan_ex(int64_t N, double W, double eps, const slepian_plan_opts *opts, slepian_plan_t *out) {
  if (!out) return SLEPIAN_EINVAL;
  int v = validate_domain(N, W, eps, opts);
  if (v != SLEPIAN_OK) return v;
  return guarded([&]() -> int {
    int dev = opts && opts->device >= 0 ? opts->device : -1;
    if (dev < 0) HIPCHK(hipGetDevice(&dev));
    DeviceGuard dg(dev);
    Plan *P = new Plan();
    P->device = dev;
    P->N = N;
    P->W = W;
    P->eps = eps;
    P->alpha = opts ? opts->alpha : 0.0;
    P->precision = opts ? opts->precision : SLEPIAN_FP32;
    P->K = (opts && opts->K > 0) ? opts->K : (int64_t)std::floor(2.0 * (double)N * W + 0.5);
    if (P->K < 1 || P->K > N - 1) {
      delete P;
      return SLEPIAN_EGAP;
    }
    hipStream_t st = nullptr;
    try {
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      build_fft_state(P, st);
      build_eigen_state(P, st);
      if (opts && opts->tune_cache) P->tune_cache = opts->tune_cache;
      if (opts && opts->tune)
        tune_plan(P, opts->tune_batch > 0 ? opts->tune_batch : kTuneBatch, opts->tune_cache, opts->tune == 2, st);
      HIPCHK(hipStreamSynchronize(st));
      (void)hipStreamDestroy(st);
    } catch (...) {
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
      delete P;
      throw;
    }
    *out = P;
    return SLEPIAN_OK;
  });
}

int slepian_plan_batch(int n, const int64_t *N, const double *W, const double *eps, const slepian_plan_opts *opts,
                       slepian_plan_t *out) {
  if (n < 0 || (n > 0 && (!N || !W || !eps || !out))) return SLEPIAN_EINVAL;
  for (int i = 0; i < n; ++i) {
    const int v = validate_domain(N[i], W[i], eps[i], opts ? &opts[i] : nullptr);
    if (v != SLEPIAN_OK) return v;
  }
  if (n == 0) return SLEPIAN_OK;
  return guarded([&]() -> int {
    int dev = opts && opts[0].device >= 0 ? opts[0].device : -1;
    if (dev < 0) HIPCHK(hipGetDevice(&dev));
    for (int i = 1; i < n; ++i)
      if (opts && opts[i].device >= 0 && opts[i].device != dev) return SLEPIAN_EINVAL;
    DeviceGuard dg(dev);
    std::vector<Plan *> Ps;
    hipStream_t st = nullptr;
    try {
      for (int i = 0; i < n; ++i) {
        Plan *P = new Plan();
        Ps.push_back(P);
        const slepian_plan_opts *o = opts ? &opts[i] : nullptr;
        P->device = dev;
        P->N = N[i];
        P->W = W[i];
        P->eps = eps[i];
        P->alpha = o ? o->alpha : 0.0;
        P->precision = o ? o->precision : SLEPIAN_FP32;
        P->K = (o && o->K > 0) ? o->K : (int64_t)std::floor(2.0 * (double)N[i] * W[i] + 0.5);
        if (P->K < 1 || P->K > N[i] - 1) throw Fail{SLEPIAN_EGAP};
      }
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      for (Plan *P : Ps) build_fft_state(P, st);
      build_eigen_states(Ps, st);
      for (int i = 0; i < n; ++i)
        if (opts && opts[i].tune_cache) Ps[i]->tune_cache = opts[i].tune_cache;
      for (int i = 0; i < n; ++i)
        if (opts && opts[i].tune)
          tune_plan(Ps[i], opts[i].tune_batch > 0 ? opts[i].tune_batch : kTuneBatch, opts[i].tune_cache,
                    opts[i].tune == 2, st);
      HIPCHK(hipStreamSynchronize(st));
      (void)hipStreamDestroy(st);
    } catch (...) {
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
      for (Plan *P : Ps) delete P;
      throw;
    }
    for (int i = 0; i < n; ++i) out[i] = Ps[i];
    return SLEPIAN_OK;
  });
}

int slepian_plan(int64_t N, double W, double eps, slepian_plan_t *out) {
  return slepian_plan_ex(N, W, eps, nullptr, out);
}

int slepian_plan_destroy(slepian_plan_t plan) {
  if (!plan) return SLEPIAN_OK;
  return guarded([&]() -> int {
    DeviceGuard dg(plan->device);
    (void)hipDeviceSynchronize();
    delete plan;
    return SLEPIAN_OK;
  });
}

int slepian_plan_info_get(slepian_plan_t P, slepian_plan_info *info) {
  if (!P || !info) return SLEPIAN_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->N = P->N;
  info->W = P->W;
  info->eps = P->eps;
  info->alpha = P->alpha;
  info->K = P->K;
  info->L = P->L;
  info->r = P->proj.r;
  info->l_first = P->u_l0 + P->proj.off;
  info->r_tik = P->tik.r;
  info->l_first_tik = P->tik.r ? P->u_l0 + P->tik.off : 0;
  info->window_lo = P->win_lo;
  info->window_hi = P->win_hi;
  info->lam_Km1 = P->lam_Km1;
  info->lam_K = P->lam_K;
  info->eps_achieved = P->eps_ach;
  info->precision = P->precision;
  info->device = P->device;
  info->row_log2 = P->g32.log2;
  info->col_log2 = P->g32.log1;
  info->cic_shape = P->g32.cic;
  info->cic_maxlog1 = P->g32.cicmax;
  info->tuned = P->tuned;
  info->tune_batch = P->tune_batch;
  info->tune_us = P->tune_us;
  return SLEPIAN_OK;
}

int slepian_plan_eigenpairs(slepian_plan_t P, int64_t *l_first, int64_t *count, double *lam_host, double *vecs,
                            int64_t ldv, int64_t cap) {
  if (!P || !l_first || !count) return SLEPIAN_EINVAL;
  *l_first = P->u_l0;
  *count = P->u_r;
  if ((lam_host || vecs) && cap < P->u_r) return SLEPIAN_ENOMEM;
  if (vecs && ldv < P->N) return SLEPIAN_EINVAL;
  if (lam_host)
    for (int64_t c = 0; c < P->u_r; ++c) lam_host[c] = P->lam[P->u_l0 - P->win_lo + c];
  if (vecs && P->u_r > 0) {
    return guarded([&]() -> int {
      DeviceGuard dg(P->device);
      HIPCHK(hipMemcpy2D(vecs, ldv * sizeof(double), P->U64, P->N * sizeof(double), P->N * sizeof(double), P->u_r,
                         hipMemcpyDeviceToDevice));
      return SLEPIAN_OK;
    });
  }
  return SLEPIAN_OK;
}

int slepian_workspace_size(slepian_plan_t P, int op, int64_t batch, size_t *bytes) {
  if (!P || !bytes || batch < 0 || op < SLEPIAN_OP_PROJECT || op > SLEPIAN_OP_MULTIBAND) return SLEPIAN_EINVAL;
  *bytes = op_workspace(P, op, batch);
  return SLEPIAN_OK;
}

int slepian_project_ex(slepian_plan_t P, int precision, const float *x, int64_t ldx, float *y, int64_t ldy,
                       int64_t batch, void *work, size_t work_bytes, void *stream) {
  if (bad_signal_args(P, x, ldx, y, ldy, batch)) return SLEPIAN_EINVAL;
  if (precision < SLEPIAN_FP32 || precision > SLEPIAN_BF16_RAW) return SLEPIAN_EINVAL;
  if (batch == 0) return SLEPIAN_OK;
  if (overlapping(x, ldx, y, ldy, P->N, batch)) return SLEPIAN_EINVAL;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t need = op_workspace(P, SLEPIAN_OP_PROJECT, batch);
    void *ws = get_ws(P, work, work_bytes, need);
    Carver cv(ws);
    ProjWs w = carve_project(P, P->proj, batch, cv, precision);
    run_fast_op(P, P->proj, 1.0f, 0.0f, x, ldx, y, ldy, batch, w, st, precision);
    return SLEPIAN_OK;
  });
}

int slepian_project_multiband(slepian_plan_t P, int nbands, const double *freqs, const float *x, int64_t ldx,
                              float *y, int64_t ldy, int64_t batch, void *work, size_t work_bytes, void *stream) {
  if (bad_signal_args(P, x, ldx, y, ldy, batch)) return SLEPIAN_EINVAL;
  BandSet bs;
  if (!parse_bands(P, nbands, freqs, bs)) return SLEPIAN_EINVAL;
  if (2 * (int64_t)nbands * batch > 32 * 65535) return SLEPIAN_EINVAL;
  if (batch == 0) return SLEPIAN_OK;
  if (overlapping(x, ldx, y, ldy, P->N, batch)) return SLEPIAN_EINVAL;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = P->N, nb = (int64_t)nbands * batch;
    void *ws = get_ws(P, work, work_bytes, op_workspace(P, SLEPIAN_OP_MULTIBAND, nb));
    Carver cv(ws);
    float *z = cv.take<float>((size_t)N * 2 * nb);
    float *pz = cv.take<float>((size_t)N * 2 * nb);
    ProjWs w = carve_project(P, P->proj, 2 * nb, cv, P->precision);
    HIPCHK(band_demod(x, ldx, N, batch, bs, z, N, st));
    run_fast_op(P, P->proj, 1.0f, 0.0f, z, N, pz, N, 2 * nb, w, st, P->precision);
    HIPCHK(band_remod(pz, N, N, batch, bs, y, ldy, st));
    return SLEPIAN_OK;
  });
}

int slepian_bands_create(slepian_plan_t P, int nbands, const double *freqs, slepian_bands_t *out) {
  if (!out) return SLEPIAN_EINVAL;
  *out = nullptr;
  BandSet bs;
  if (!parse_bands(P, nbands, freqs, bs)) return SLEPIAN_EINVAL;
  if (P->proj.r > kMbMaxRank) return SLEPIAN_ENOTSUP;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    auto *B = new slepian_bands_s;
    B->P = P;
    B->device = P->device;
    B->bs = bs;
    hipStream_t st = nullptr;
    try {
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      const int64_t L = P->L, N = P->N;
      // spectrum of the band-sum kernel's circulant embedding, as the plan's own (FP64 transform)
      const FftGeom gen64 = generic_twin(P->g64);
      {
        DBuf<double> c(L);
        DBuf<cpx<double>> spec(L);
        HIPCHK(band_embed(c.p, L, N, P->W, bs, st));
        HIPCHK(fft_forward_real64(c.p, gen64, P->tb64, spec.p, st));
        B->chat32 = dalloc<float>(L);
        HIPCHK(spectrum_relayout<float>(spec.p, gen64, B->chat32, P->g32, st));
        HIPCHK(hipStreamSynchronize(st));
      }
      B->ldm = mb_ldm(N);
      B->M = dalloc<float>((size_t)band_table_rows(bs.J) * B->ldm);
      HIPCHK(band_table(B->M, B->ldm, N, bs, st));
      HIPCHK(hipStreamSynchronize(st));
      B->mode = P->precision == SLEPIAN_FP32 ? 0 : 1;
      B->u = mb_layout(P, B->mode);
      (void)hipStreamDestroy(st);
    } catch (...) {
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
      delete B;
      throw;
    }
    *out = B;
    return SLEPIAN_OK;
  });
}

int slepian_bands_destroy(slepian_bands_t B) {
  if (!B) return SLEPIAN_OK;
  return guarded([&]() -> int {
    DeviceGuard dg(B->device);
    (void)hipDeviceSynchronize();
    delete B;
    return SLEPIAN_OK;
  });
}

int slepian_bands_workspace_size(slepian_bands_t B, int64_t batch, size_t *bytes) {
  if (!B || !bytes || batch < 0) return SLEPIAN_EINVAL;
  *bytes = bands_workspace(B, batch);
  return SLEPIAN_OK;
}

namespace {

// y = sum_i w_i Re(E_i P~ E_i^* x) for the prepared bands, with the band
// sum's workspace at ws (bands_workspace bytes); y may equal x.
void bands_apply(slepian_bands_s *B, const float *x, int64_t ldx, float *y, int64_t ldy, int64_t batch, void *ws,
                 hipStream_t st) {
  Plan *P = B->P;
  const int64_t N = P->N;
  const int r = (int)P->proj.r;
  const MbShape sh = mb_shape(N, batch, r, B->bs.J);
  Carver cv(ws);
  const int64_t pairs = (batch + 1) / 2;
  const int64_t slice = (int64_t)conv_workspace_pairs(P->g32, pairs, sizeof(cpx<float>), slice_budget());
  cpx<float> *Z = P->g32.single() ? nullptr : cv.take<cpx<float>>((size_t)slice * (size_t)P->L);
  MbWs mw;
  if (r > 0) mw = mb_carve(sh, batch, cv.take<char>(mb_workspace_bytes(sh, batch)));
  // the coefficients read x before the product writes y (which may be x)
  HIPCHK(mb_coeffs(B->mode, x, ldx, N, batch, B->u, r, P->proj.d32, B->M, B->ldm, B->bs, sh, mw, st));
  FftTables<float> tb = P->tb32;
  tb.chat = B->chat32;
  HIPCHK(conv_apply<float>(x, ldx, y, ldy, N, batch, P->g32, tb, 1.0f, 0.0f, Corr<float>(), Z, slice, st));
  HIPCHK(mb_apply(B->mode, y, ldy, N, batch, B->u, r, B->M, B->ldm, sh, mw, st));
}

int64_t span_ld(int64_t N) { return (N + 63) / 64 * 64; }

// The span projection's workspace: the band sum's, then r, p and A p
// (leading dimension span_ld(N)), the dot products' chunk partials and one
// iteration record per signal.
size_t bands_span_workspace(const slepian_bands_s *B, int64_t b) {
  const int64_t N = B->P->N;
  Carver cv(nullptr);
  cv.take<char>(bands_workspace(B, b));
  cv.take<float>((size_t)span_ld(N) * b * 3);
  cv.take<double>((size_t)cg_nchunks(N) * b);
  cv.take<CgState>((size_t)b);
  return cv.off + 256;
}

}  // namespace

int slepian_project_bands(slepian_bands_t B, const float *x, int64_t ldx, float *y, int64_t ldy, int64_t batch,
                          void *work, size_t work_bytes, void *stream) {
  if (!B) return SLEPIAN_EINVAL;
  Plan *P = B->P;
  if (bad_signal_args(P, x, ldx, y, ldy, batch)) return SLEPIAN_EINVAL;
  if (batch == 0) return SLEPIAN_OK;
  if (overlapping(x, ldx, y, ldy, P->N, batch)) return SLEPIAN_EINVAL;
  const int r = (int)P->proj.r;
  const MbShape sh = mb_shape(P->N, batch, r, B->bs.J);
  if (r > 0 && !mb_ok(sh, P->N, batch, r)) return SLEPIAN_ENOTSUP;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    void *ws = get_ws(P, work, work_bytes, bands_workspace(B, batch));
    bands_apply(B, x, ldx, y, ldy, batch, ws, (hipStream_t)stream);
    return SLEPIAN_OK;
  });
}

int slepian_bands_span_workspace_size(slepian_bands_t B, int64_t batch, size_t *bytes) {
  if (!B || !bytes || batch < 0) return SLEPIAN_EINVAL;
  *bytes = bands_span_workspace(B, batch);
  return SLEPIAN_OK;
}

int slepian_project_bands_span(slepian_bands_t B, const float *x, int64_t ldx, float *y, int64_t ldy,
                               int64_t batch, double tol, int max_iter, void *work, size_t work_bytes, void *stream,
                               int *iters) {
  if (!B) return SLEPIAN_EINVAL;
  Plan *P = B->P;
  if (bad_signal_args(P, x, ldx, y, ldy, batch)) return SLEPIAN_EINVAL;
  if (tol == 0.0) tol = std::max(P->eps, kSpanMinTol);
  if (!(tol >= kSpanMinTol && tol < 0.5) || max_iter < 1 || max_iter > 1000) return SLEPIAN_EINVAL;
  if (batch == 0) return SLEPIAN_OK;
  if (overlapping(x, ldx, y, ldy, P->N, batch)) return SLEPIAN_EINVAL;
  const int r = (int)P->proj.r;
  const MbShape sh = mb_shape(P->N, batch, r, B->bs.J);
  if (r > 0 && !mb_ok(sh, P->N, batch, r)) return SLEPIAN_ENOTSUP;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = P->N, ldw = span_ld(N);
    void *ws = get_ws(P, work, work_bytes, bands_span_workspace(B, batch));
    Carver cv(ws);
    void *wa = cv.take<char>(bands_workspace(B, batch));
    float *rv = cv.take<float>((size_t)ldw * batch);
    float *pv = cv.take<float>((size_t)ldw * batch);
    float *ap = cv.take<float>((size_t)ldw * batch);
    double *part = cv.take<double>((size_t)cg_nchunks(N) * batch);
    CgState *state = cv.take<CgState>((size_t)batch);
    // r = A x (x is not read again, so y may be x), z = 0, p = r
    bands_apply(B, x, ldx, rv, ldw, batch, wa, st);
    HIPCHK(cg_dot(rv, ldw, rv, ldw, N, batch, part, st));
    HIPCHK(cg_init(part, N, batch, tol, state, st));
    HIPCHK(fill_zero_rows(y, ldy, N, batch, st));
    HIPCHK(copy_rows(rv, ldw, pv, ldw, N, batch, st));
    std::vector<CgState> hs((size_t)batch);
    bool any = true;
    for (int k = 0; k <= max_iter; ++k) {
      HIPCHK(hipMemcpyAsync(hs.data(), state, (size_t)batch * sizeof(CgState), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      any = false;
      for (const CgState &q : hs) {
        // a NaN or Inf in x shows up in ||A x||^2 and the residual norms
        if (!std::isfinite(q.nb2) || !std::isfinite(q.rr)) return SLEPIAN_ENONFINITE;
        any = any || q.active;
      }
      if (!any || k == max_iter) break;
      bands_apply(B, pv, ldw, ap, ldw, batch, wa, st);
      HIPCHK(cg_dot(pv, ldw, ap, ldw, N, batch, part, st));
      HIPCHK(cg_alpha(part, N, batch, state, st));
      HIPCHK(cg_update(y, ldy, rv, pv, ap, ldw, N, batch, state, part, st));
      HIPCHK(cg_beta(part, N, batch, tol, state, st));
      HIPCHK(cg_direction(pv, rv, ldw, N, batch, state, st));
    }
    if (iters)
      for (int64_t s = 0; s < batch; ++s) iters[s] = hs[(size_t)s].iters;
    return any ? SLEPIAN_ENOCONV : SLEPIAN_OK;
  });
}

// ---------------------------------------------------------------------------
// Fast factorization S_K S_K^T ~= T1 T2^T (Section 1.3, Theorem 1)
// ---------------------------------------------------------------------------

struct slepian_factor_s {
  slepian_plan_s *P = nullptr;
  int device = 0;
  int kf = 0;                 // 2NW', the odd integer nearest to 2NW
  int64_t r1 = 0, r = 0;      // columns of the Theorem 1 factor and of the transition set
  int64_t p = 0;              // subspace size the setup converged with
  double defl = 0;            // estimated norm of B - F F^* deflated by the kept pairs
  double mu_drop = 0;         // largest |Ritz value| left out (<= eps)
  double ritz_res = 0;        // largest ||T v_j - mu_j v_j|| of the kept pairs
  int method = SLEPIAN_FACTOR_THEOREM1;
  int rH = 0, rA = 0, rB = 0; // Theorem 1's construction: Hilbert-factor columns, series terms
  float *U = nullptr;         // N x (r1 + r), leading dimension ldu: compression [L2 | U_T]
  float *Urec = nullptr;      // recovery [L1 | U_T] when it differs from U (THEOREM1), else null
  int64_t ldu = 0;
  float *w = nullptr;         // r1 + r weights: [mu | d] (EIG) or [1 | d] (THEOREM1)
  int mode = 0;               // matrix mode of the coefficient products
  void *ctile = nullptr;      // the recovery matrix laid out for the fused inverse column pass (or null)
  std::vector<double> mu;
  const float *rec() const { return Urec ? Urec : U; }
  ~slepian_factor_s() {
    dfree(U);
    dfree(Urec);
    dfree(w);
    dfree(ctile);
  }
};

namespace {

// 2NW': nearest odd integer to 2NW, ties (2NW an even integer) upward.
int factor_kf(int64_t N, double W) {
  const double v = 2.0 * (double)N * W;
  int64_t lo = (int64_t)std::floor(v);
  if (lo % 2 == 0) lo -= 1;
  const int64_t hi = lo + 2;
  return (int)((v - (double)lo) < ((double)hi - v) ? lo : hi);
}

struct RocHandle {
  rocblas_handle h = nullptr;
  explicit RocHandle(hipStream_t st) {
    if (rocblas_create_handle(&h) != rocblas_status_success) throw Fail{SLEPIAN_EHIP};
    if (rocblas_set_stream(h, st) != rocblas_status_success) throw Fail{SLEPIAN_EHIP};
  }
  ~RocHandle() {
    if (h) (void)rocblas_destroy_handle(h);
  }
};

#define ROCCHK(call)                                             \
  do {                                                           \
    if ((call) != rocblas_status_success) throw Fail{SLEPIAN_EHIP}; \
  } while (0)

size_t factor_workspace(const slepian_factor_s *F, int64_t b) {
  const Plan *P = F->P;
  Carver cv(nullptr);
  const int64_t pairs = (b + 1) / 2;
  cv.take<cpx<float>>((size_t)pairs * F->kf);
  const int64_t slice = (int64_t)conv_workspace_pairs(P->g32, pairs, sizeof(cpx<float>), slice_budget());
  if (!P->g32.single()) cv.take<cpx<float>>((size_t)slice * (size_t)P->L);
  const int rt = (int)(F->r1 + F->r);
  if (rt > 0) {
    cv.take<float>((size_t)corr_nchunks(P->N, b, rt) * corr_rpad(rt) * b);
    cv.take<float>((size_t)b * corr_rpad(rt));
  }
  return cv.off;
}

struct FactorWs {
  cpx<float> *Zb = nullptr, *Z = nullptr;
  int64_t slice = 0;
  float *part = nullptr, *dC = nullptr;
};

FactorWs carve_factor(const slepian_factor_s *F, int64_t b, void *base) {
  const Plan *P = F->P;
  Carver cv(base);
  FactorWs w;
  const int64_t pairs = (b + 1) / 2;
  w.Zb = cv.take<cpx<float>>((size_t)pairs * F->kf);
  w.slice = (int64_t)conv_workspace_pairs(P->g32, pairs, sizeof(cpx<float>), slice_budget());
  if (!P->g32.single()) w.Z = cv.take<cpx<float>>((size_t)w.slice * (size_t)P->L);
  const int rt = (int)(F->r1 + F->r);
  if (rt > 0) {
    w.part = cv.take<float>((size_t)corr_nchunks(P->N, b, rt) * corr_rpad(rt) * b);
    w.dC = cv.take<float>((size_t)b * corr_rpad(rt));
  }
  return w;
}

// Estimate of the largest |eigenvalue| of (I - V V^T) T (I - V V^T), T the
// FP64 product with spectrum tbt and V (N x r1, orthonormal columns) the kept
// eigenvectors: kDeflSteps block power steps on 8 +-1 columns, the block
// re-orthonormalised (Householder QR) before each product and V's component
// removed before and after it; the largest column norm of the last deflated
// product.
double deflated_norm(const Plan *P, const FftTables<double> &tbt, const B64Ws &bw, const double *V, int64_t r1,
                     RocHandle &rh, hipStream_t st) {
  constexpr int kDeflSteps = 6;
  constexpr int64_t q = 8;
  const int64_t N = P->N;
  DBuf<double> G((size_t)N * q), Y((size_t)N * q), tau(q), Cq((size_t)std::max<int64_t>(r1, 1) * q), nrm(q),
      part((size_t)q * kNormParts);
  const double one = 1.0, zero = 0.0, mone = -1.0;
  auto deflate = [&](double *X) {
    if (r1 == 0) return;
    ROCCHK(rocblas_dgemm(rh.h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)r1, (rocblas_int)q,
                         (rocblas_int)N, &one, V, (rocblas_int)N, X, (rocblas_int)N, &zero, Cq.p, (rocblas_int)r1));
    ROCCHK(rocblas_dgemm(rh.h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)N, (rocblas_int)q,
                         (rocblas_int)r1, &mone, V, (rocblas_int)N, Cq.p, (rocblas_int)r1, &one, X, (rocblas_int)N));
  };
  HIPCHK(rademacher(G.p, N, N, q, 0xdef1a7edull, st));
  for (int it = 0; it < kDeflSteps; ++it) {
    deflate(G.p);
    ROCCHK(rocsolver_dgeqrf(rh.h, (rocblas_int)N, (rocblas_int)q, G.p, (rocblas_int)N, tau.p));
    ROCCHK(rocsolver_dorgqr(rh.h, (rocblas_int)N, (rocblas_int)q, (rocblas_int)q, G.p, (rocblas_int)N, tau.p));
    deflate(G.p);
    HIPCHK(conv_apply<double>(G.p, N, Y.p, N, N, q, P->g64, tbt, 1.0, 0.0, Corr<double>(), bw.Z, bw.slice, st));
    deflate(Y.p);
    std::swap(G.p, Y.p);
  }
  HIPCHK(col_norms(G.p, N, N, q, nrm.p, part.p, st));
  std::vector<double> h(q);
  HIPCHK(hipMemcpyAsync(h.data(), nrm.p, (size_t)q * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double m = 0;
  for (double v : h) m = std::max(m, v);
  return m;
}

// V, mu with B - F F^* ~= V diag(mu) V^T over the eigenpairs with |mu| > eps:
// subspace iteration on a +-1 start block of p columns with the FP64 product
// (Toeplitz kernel t of B - F F^*), Householder QR after every product, then
// a Rayleigh-Ritz step.  p doubles until at least 24 Ritz values fall at or
// below eps, every kept pair's residual ||T v - mu v|| is at most eps / 4,
// and the operator deflated by the kept vectors has norm at most eps
// (deflated_norm).
void factor_setup(slepian_factor_s *F, hipStream_t st) {
  Plan *P = F->P;
  const int64_t N = P->N, L = P->L;
  // spectrum of t's circulant embedding in the FP64 product's layout
  const FftGeom gen64 = generic_twin(P->g64);
  DBuf<double> chat(L);
  {
    DBuf<double> c(L);
    DBuf<cpx<double>> spec(L);
    HIPCHK(diff_embed(c.p, L, N, P->W, F->kf, st));
    HIPCHK(fft_forward_real64(c.p, gen64, P->tb64, spec.p, st));
    HIPCHK(spectrum_relayout<double>(spec.p, gen64, chat.p, P->g64, st));
  }
  FftTables<double> tbt = P->tb64;
  tbt.chat = chat.p;
  RocHandle rh(st);
  constexpr int kIters = 6, kMargin = 24;
  int64_t p = std::min<int64_t>(96, N - 1);
  for (;;) {
    DBuf<double> Q((size_t)N * p), Y((size_t)N * p), tau(p), H((size_t)p * p), D(p), E(p);
    DBuf<int> info(1);
    Carver mc(nullptr);
    carve_b64(P, p, mc);
    DBuf<char> ws(std::max<size_t>(mc.off, 256));
    Carver cv(ws.p);
    const B64Ws bw = carve_b64(P, p, cv);
    HIPCHK(rademacher(Q.p, N, N, p, 0x5eed5eedull, st));
    for (int it = 0; it <= kIters; ++it) {
      HIPCHK(conv_apply<double>(Q.p, N, Y.p, N, N, p, P->g64, tbt, 1.0, 0.0, Corr<double>(), bw.Z, bw.slice, st));
      if (it == kIters) break;
      ROCCHK(rocsolver_dgeqrf(rh.h, (rocblas_int)N, (rocblas_int)p, Y.p, (rocblas_int)N, tau.p));
      ROCCHK(rocsolver_dorgqr(rh.h, (rocblas_int)N, (rocblas_int)p, (rocblas_int)p, Y.p, (rocblas_int)N, tau.p));
      std::swap(Q.p, Y.p);
    }
    // H = Q^T (T Q), its eigenpairs (ascending), Ritz vectors Q Z
    const double one = 1.0, zero = 0.0;
    ROCCHK(rocblas_dgemm(rh.h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)p, (rocblas_int)p,
                         (rocblas_int)N, &one, Q.p, (rocblas_int)N, Y.p, (rocblas_int)N, &zero, H.p,
                         (rocblas_int)p));
    ROCCHK(rocsolver_dsyevd(rh.h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)p, H.p, (rocblas_int)p,
                            D.p, E.p, info.p));
    std::vector<double> d(p), z((size_t)p * p);
    int inf = 0;
    HIPCHK(hipMemcpyAsync(d.data(), D.p, p * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(z.data(), H.p, (size_t)p * p * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&inf, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (inf != 0) throw Fail{SLEPIAN_ENOCONV};
    std::vector<int64_t> keep;
    double drop = 0;
    for (int64_t i = 0; i < p; ++i) {
      if (std::fabs(d[i]) > P->eps) keep.push_back(i);
      else drop = std::max(drop, std::fabs(d[i]));
    }
    if (p - (int64_t)keep.size() < kMargin) {
      if (p >= std::min<int64_t>(1024, N - 1)) throw Fail{SLEPIAN_ENOCONV};
      p = std::min<int64_t>(2 * p, std::min<int64_t>(1024, N - 1));
      continue;
    }
    std::stable_sort(keep.begin(), keep.end(), [&](int64_t a, int64_t b) { return std::fabs(d[a]) > std::fabs(d[b]); });
    const int64_t r1 = (int64_t)keep.size();
    std::vector<double> mu(r1), zs((size_t)p * std::max<int64_t>(r1, 1));
    for (int64_t j = 0; j < r1; ++j) {
      mu[j] = d[keep[j]];
      std::copy(z.begin() + keep[j] * p, z.begin() + (keep[j] + 1) * p, zs.begin() + j * p);
    }
    // Ritz vectors V = Q Z, signed; their residuals ||T v_j - mu_j v_j||
    // checked against eps / 4 (else a wider block)
    std::unique_ptr<DBuf<double>> V;
    double res = 0;
    if (r1 > 0) {
      V.reset(new DBuf<double>((size_t)N * r1));
      DBuf<double> Zs((size_t)p * r1), R((size_t)N * r1), mud(r1), nrm(r1), part((size_t)r1 * kNormParts);
      HIPCHK(hipMemcpyAsync(Zs.p, zs.data(), (size_t)p * r1 * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(mud.p, mu.data(), (size_t)r1 * sizeof(double), hipMemcpyHostToDevice, st));
      ROCCHK(rocblas_dgemm(rh.h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)N, (rocblas_int)r1,
                           (rocblas_int)p, &one, Q.p, (rocblas_int)N, Zs.p, (rocblas_int)p, &zero, V->p,
                           (rocblas_int)N));
      HIPCHK(sign_fix_cols(V->p, N, N, r1, st));
      HIPCHK(conv_apply<double>(V->p, N, R.p, N, N, r1, P->g64, tbt, 1.0, 0.0, Corr<double>(), bw.Z, bw.slice, st));
      HIPCHK(ritz_residual(R.p, V->p, mud.p, N, N, r1, st));
      HIPCHK(col_norms(R.p, N, N, r1, nrm.p, part.p, st));
      std::vector<double> h(r1);
      HIPCHK(hipMemcpyAsync(h.data(), nrm.p, (size_t)r1 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (double v : h) res = std::max(res, v);
      if (!(res <= 0.25 * P->eps)) {
        if (p >= std::min<int64_t>(1024, N - 1)) throw Fail{SLEPIAN_ENOCONV};
        p = std::min<int64_t>(2 * p, std::min<int64_t>(1024, N - 1));
        continue;
      }
    }
    // A posteriori: no eigenvalue with |mu| > eps may lie outside span(V).
    // Block power steps on the deflated operator (I - V V^T) T (I - V V^T)
    // from a fresh +-1 block (QR between steps); its largest column norm
    // after the last product estimates the largest |mu| left out.  Above eps
    // the block was too narrow: widen it, or ENOCONV at the cap.
    const double defl = deflated_norm(P, tbt, bw, V ? V->p : nullptr, r1, rh, st);
    if (!(defl <= P->eps)) {
      if (p >= std::min<int64_t>(1024, N - 1)) throw Fail{SLEPIAN_ENOCONV};
      p = std::min<int64_t>(2 * p, std::min<int64_t>(1024, N - 1));
      continue;
    }
    F->r1 = r1;
    F->p = p;
    F->mu_drop = drop;
    F->ritz_res = res;
    F->defl = defl;
    F->mu = mu;
    const int64_t rt = r1 + F->r;
    F->ldu = (N + 3) / 4 * 4;
    F->U = dalloc<float>((size_t)F->ldu * std::max<int64_t>(rt, 1));
    if (r1 > 0) {
      HIPCHK(cast_f64_to_f32(V->p, N, F->U, F->ldu, N, r1, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    if (F->r > 0)
      HIPCHK(copy_f32(P->U32 + P->proj.off * P->ldu, P->ldu, F->U + r1 * F->ldu, F->ldu, N, F->r, st));
    std::vector<float> w32(std::max<int64_t>(rt, 1));
    for (int64_t j = 0; j < r1; ++j) w32[j] = (float)F->mu[j];
    for (int64_t j = 0; j < F->r; ++j) w32[r1 + j] = (float)P->proj.d[j];
    F->w = dalloc<float>(w32.size());
    HIPCHK(hipMemcpyAsync(F->w, w32.data(), w32.size() * sizeof(float), hipMemcpyHostToDevice, st));
    const FftGeom &g = P->g32;
    if (rt > 0 && !g.single() && colinv_corr_tiled(g)) {
      F->ctile = dalloc<char>(corr_tile_bytes(g.log1, g.log2, (int)rt, F->mode));
      HIPCHK(build_corr_tile(F->U, F->ldu, (int)N, (int)rt, g.log1, g.log2, F->mode, F->ctile, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    return;
  }
}

// ---- Theorem 1's construction (Section 2): host-side constants ----

// Arithmetic-geometric mean of 1 and kc with the half-differences c_n
// (c_0 = sqrt(1 - kc^2)), at most 64 halvings.
void agm_steps(double kc, std::vector<double> &a, std::vector<double> &c) {
  a.assign(1, 1.0);
  c.assign(1, std::sqrt((1.0 - kc) * (1.0 + kc)));
  double b = kc;
  for (int i = 0; i < 64 && c.back() > 4e-16 * a.back(); ++i) {
    const double an = a.back();
    a.push_back(0.5 * (an + b));
    c.push_back(0.5 * (an - b));
    b = std::sqrt(an * b);
  }
}

// Jacobi dn(u, tau), tau = sqrt(1 - kc^2), by the descending Landen scheme.
double jacobi_dn(double u, const std::vector<double> &a, const std::vector<double> &c) {
  const int n = (int)a.size() - 1;
  if (n == 0) return 1.0;
  double phi = std::ldexp(a[n] * u, n), prev = phi;
  for (int k = n; k >= 1; --k) {
    prev = phi;
    phi = 0.5 * (phi + std::asin(c[k] * std::sin(phi) / a[k]));
  }
  return std::cos(phi) / std::cos(prev - phi);
}

// zeta(s) for s >= 2 by Euler-Maclaurin summation with 16 leading terms and
// five Bernoulli corrections.
double zeta_em(double s) {
  constexpr int M = 16;
  double z = 0.0;
  for (int n = 1; n < M; ++n) z += std::pow((double)n, -s);
  const double m = (double)M;
  z += std::pow(m, 1.0 - s) / (s - 1.0) + 0.5 * std::pow(m, -s);
  static const double b2j[5] = {1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66};
  double rising = s, fact = 2.0;  // s (s+1) ... (s+2j-2) and (2j)!
  for (int j = 1; j <= 5; ++j) {
    z += b2j[j - 1] / fact * rising * std::pow(m, -s - 2.0 * j + 1.0);
    rising *= (s + 2.0 * j - 1.0) * (s + 2.0 * j);
    fact *= (2.0 * j + 1.0) * (2.0 * j + 2.0);
  }
  return z;
}

double binom(int n, int k) {
  double v = 1.0;
  for (int i = 1; i <= k; ++i) v = v * (double)(n - k + i) / (double)i;
  return std::round(v);
}

struct Thm1Consts {
  int rH = 0, rA = 0, rB = 0;
  std::vector<double> prm;  // [shifts | C_A | C_B]
};

// delta_H = 4 pi eps / 15, delta_A = delta_B = 7 eps / 30 ("Putting it all
// together"); rH from Lemma 2 with kappa = 2N - 1, delta = delta_H / pi;
// shifts p_j = b dn((2j - 1)/(2 rH) I(tau), tau) on [a, b] = [1/2, N - 1/2]
// (the appendix's remark on the optimal parameters); C_A from the zeta
// coefficients 1 - (1 - 2^{-(2k-1)}) zeta(2k) of A1's odd series, C_B from the
// sine series of B0 with theta = pi (W - W') N, both expanded binomially in
// the centred index u = (n - (N-1)/2) / N.
Thm1Consts theorem1_consts(int64_t N, double W, double eps, int kf) {
  Thm1Consts t;
  const double dH = 4.0 * M_PI * eps / 15.0, dA = 7.0 * eps / 30.0, dB = dA;
  t.rH = (int)std::ceil(std::log(8.0 * (double)N - 4.0) * std::log(4.0 * M_PI / dH) / (M_PI * M_PI));
  t.rA = (int)std::ceil(std::log(2.0 / (3.0 * M_PI * dA)) / (2.0 * std::log(2.0)));
  t.rB = (int)std::ceil(std::log(3.0 / (2.0 * dB)) / (2.0 * std::log(6.0 / M_PI)));
  const double a = 0.5, b = (double)N - 0.5;
  std::vector<double> ag, cg;
  agm_steps(a / b, ag, cg);
  const double K = M_PI / (2.0 * ag.back());
  for (int j = 1; j <= t.rH; ++j) t.prm.push_back(b * jacobi_dn((2.0 * j - 1.0) / (2.0 * t.rH) * K, ag, cg));
  const int na = 2 * t.rA, nb = 2 * t.rB - 1;
  const size_t oa = t.prm.size();
  t.prm.resize(oa + (size_t)na * na + (size_t)nb * nb, 0.0);
  const double scale = 2.0 / ((double)N * M_PI);
  for (int k = 1; k <= t.rA; ++k) {
    const double ck = 1.0 - (1.0 - std::ldexp(1.0, -(2 * k - 1))) * zeta_em(2.0 * k);
    const int pdeg = 2 * k - 1;
    for (int i = 0; i <= pdeg; ++i)
      t.prm[oa + (size_t)i * na + (pdeg - i)] = scale * ck * binom(pdeg, i) * (((pdeg - i) & 1) ? -1.0 : 1.0);
  }
  const size_t ob = oa + (size_t)na * na;
  const double Wp = (double)kf / (2.0 * (double)N);
  const double theta = M_PI * (W - Wp) * (double)N;
  double pw = theta, fact = 1.0;  // theta^{2k+1} and (2k+1)!
  for (int k = 0; k < t.rB; ++k) {
    const double coef = scale * ((k & 1) ? -1.0 : 1.0) * pw / fact;
    const int pdeg = 2 * k;
    for (int i = 0; i <= pdeg; ++i)
      t.prm[ob + (size_t)i * nb + (pdeg - i)] = coef * binom(pdeg, i) * (((pdeg - i) & 1) ? -1.0 : 1.0);
    pw *= theta * theta;
    fact *= (2.0 * k + 2.0) * (2.0 * k + 3.0);
  }
  return t;
}

// L1, L2 by the construction; weights [1 | d]; the recovery matrix's tile.
void factor_setup_theorem1(slepian_factor_s *F, hipStream_t st) {
  Plan *P = F->P;
  const int64_t N = P->N;
  const Thm1Consts t = theorem1_consts(N, P->W, P->eps, F->kf);
  F->rH = t.rH;
  F->rA = t.rA;
  F->rB = t.rB;
  const int64_t r1 = 2 * (2 * (int64_t)t.rH + 2 * t.rA + 2 * t.rB - 1);
  F->r1 = r1;
  const int64_t rt = r1 + F->r;
  F->ldu = (N + 3) / 4 * 4;
  F->U = dalloc<float>((size_t)F->ldu * rt);
  F->Urec = dalloc<float>((size_t)F->ldu * rt);
  {
    DBuf<double> prm(t.prm.size());
    HIPCHK(hipMemcpyAsync(prm.p, t.prm.data(), t.prm.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(theorem1_rows(N, F->kf, P->W, t.rH, t.rA, t.rB, prm.p, F->U, F->Urec, F->ldu, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (F->r > 0) {
    HIPCHK(copy_f32(P->U32 + P->proj.off * P->ldu, P->ldu, F->U + r1 * F->ldu, F->ldu, N, F->r, st));
    HIPCHK(copy_f32(P->U32 + P->proj.off * P->ldu, P->ldu, F->Urec + r1 * F->ldu, F->ldu, N, F->r, st));
  }
  std::vector<float> w32(std::max<int64_t>(rt, 1), 1.0f);
  for (int64_t j = 0; j < F->r; ++j) w32[r1 + j] = (float)P->proj.d[j];
  F->w = dalloc<float>(w32.size());
  HIPCHK(hipMemcpyAsync(F->w, w32.data(), w32.size() * sizeof(float), hipMemcpyHostToDevice, st));
  const FftGeom &g = P->g32;
  if (rt > 0 && !g.single() && colinv_corr_tiled(g)) {
    F->ctile = dalloc<char>(corr_tile_bytes(g.log1, g.log2, (int)rt, F->mode));
    HIPCHK(build_corr_tile(F->Urec, F->ldu, (int)N, (int)rt, g.log1, g.log2, F->mode, F->ctile, st));
  }
  HIPCHK(hipStreamSynchronize(st));
}

bool bad_factor_args(const slepian_factor_s *F, const void *in, int64_t ldin, int64_t rows_in, const void *out,
                     int64_t ldout, int64_t rows_out, int64_t batch) {
  if (!F || batch < 0 || batch > 32 * (int64_t)65535) return true;
  if (batch == 0) return false;
  return !in || !out || ldin < rows_in || ldout < rows_out;
}

bool factor_overlap(const void *a, int64_t lda, int64_t rows_a, const void *b, int64_t ldb, int64_t rows_b,
                    int64_t batch) {
  const char *a0 = static_cast<const char *>(a), *b0 = static_cast<const char *>(b);
  const char *a1 = a0 + ((batch - 1) * lda + rows_a) * (int64_t)sizeof(float);
  const char *b1 = b0 + ((batch - 1) * ldb + rows_b) * (int64_t)sizeof(float);
  return a0 < b1 && b0 < a1;
}

}  // namespace

int slepian_factor_create(slepian_plan_t P, slepian_factor_t *out) {
  return slepian_factor_create_ex(P, SLEPIAN_FACTOR_THEOREM1, out);
}

int slepian_factor_create_ex(slepian_plan_t P, int method, slepian_factor_t *out) {
  if (!out) return SLEPIAN_EINVAL;
  *out = nullptr;
  if (!P) return SLEPIAN_EINVAL;
  if (method != SLEPIAN_FACTOR_THEOREM1 && method != SLEPIAN_FACTOR_EIG) return SLEPIAN_EINVAL;
  if (!dft_bins_ok(P->g32, P->N) || P->N > ((int64_t)1 << 20)) return SLEPIAN_ENOTSUP;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    auto *F = new slepian_factor_s;
    F->P = P;
    F->device = P->device;
    F->kf = factor_kf(P->N, P->W);
    F->r = P->proj.r;
    F->mode = P->precision == SLEPIAN_FP32 ? 0 : 1;
    F->method = method;
    hipStream_t st = nullptr;
    try {
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      if (method == SLEPIAN_FACTOR_THEOREM1) factor_setup_theorem1(F, st);
      else factor_setup(F, st);
      (void)hipStreamDestroy(st);
    } catch (...) {
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
      delete F;
      throw;
    }
    *out = F;
    return SLEPIAN_OK;
  });
}

int slepian_factor_destroy(slepian_factor_t F) {
  if (!F) return SLEPIAN_OK;
  return guarded([&]() -> int {
    DeviceGuard dg(F->device);
    (void)hipDeviceSynchronize();
    delete F;
    return SLEPIAN_OK;
  });
}

int slepian_factor_info(slepian_factor_t F, slepian_factor_info_t *info) {
  if (!F || !info) return SLEPIAN_EINVAL;
  info->kf = F->kf;
  info->r1 = F->r1;
  info->r = F->r;
  info->kprime = F->kf + F->r1 + F->r;
  info->subspace = F->p;
  info->deflated_norm = F->defl;
  info->mu_dropped = F->mu_drop;
  info->ritz_residual = F->ritz_res;
  info->method = F->method;
  info->r_h = F->rH;
  info->r_a = F->rA;
  info->r_b = F->rB;
  return SLEPIAN_OK;
}

int slepian_factor_mu(slepian_factor_t F, double *mu, int64_t n) {
  if (!F) return SLEPIAN_EINVAL;
  if (F->method != SLEPIAN_FACTOR_EIG) return SLEPIAN_ENOTSUP;
  if ((n > 0 && !mu) || n < F->r1) return SLEPIAN_EINVAL;
  std::copy(F->mu.begin(), F->mu.end(), mu);
  return SLEPIAN_OK;
}

int slepian_factor_workspace_size(slepian_factor_t F, int64_t batch, size_t *bytes) {
  if (!F || !bytes || batch < 0) return SLEPIAN_EINVAL;
  *bytes = factor_workspace(F, batch);
  return SLEPIAN_OK;
}

int slepian_factor_compress(slepian_factor_t F, const float *x, int64_t ldx, float *c, int64_t ldc, int64_t batch,
                            void *work, size_t work_bytes, void *stream) {
  if (!F) return SLEPIAN_EINVAL;
  Plan *P = F->P;
  const int64_t kp = F->kf + F->r1 + F->r;
  if (bad_factor_args(F, x, ldx, P->N, c, ldc, kp, batch)) return SLEPIAN_EINVAL;
  if (batch == 0) return SLEPIAN_OK;
  if (factor_overlap(x, ldx, P->N, c, ldc, kp, batch)) return SLEPIAN_EINVAL;
  return guarded([&]() -> int {
    DeviceGuard dg(F->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = P->N;
    void *ws = get_ws(P, work, work_bytes, factor_workspace(F, batch));
    const FactorWs w = carve_factor(F, batch, ws);
    // F_r^T x: length-N DFT bins of signal pairs, then the real coefficients
    HIPCHK(dft_bins_fwd(x, ldx, N, batch, P->g32, P->tb32, w.Z, w.slice, w.Zb, F->kf, st));
    HIPCHK(bins_unpack(w.Zb, F->kf, N, batch, c, ldc, st));
    // [V U_T]^T x on the matrix cores, chunk partials summed in a fixed order
    const int rt = (int)(F->r1 + F->r);
    if (rt > 0) {
      HIPCHK(corr_partial_mfma(F->mode, x, ldx, N, batch, F->U, F->ldu, rt, w.part, st));
      HIPCHK(corr_sum_mfma(w.part, N, batch, rt, c + F->kf, ldc, st));
    }
    return SLEPIAN_OK;
  });
}

int slepian_factor_recover(slepian_factor_t F, const float *c, int64_t ldc, float *y, int64_t ldy, int64_t batch,
                           void *work, size_t work_bytes, void *stream) {
  if (!F) return SLEPIAN_EINVAL;
  Plan *P = F->P;
  const int64_t kp = F->kf + F->r1 + F->r;
  if (bad_factor_args(F, c, ldc, kp, y, ldy, P->N, batch)) return SLEPIAN_EINVAL;
  if (batch == 0) return SLEPIAN_OK;
  if (factor_overlap(c, ldc, kp, y, ldy, P->N, batch)) return SLEPIAN_EINVAL;
  return guarded([&]() -> int {
    DeviceGuard dg(F->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = P->N;
    void *ws = get_ws(P, work, work_bytes, factor_workspace(F, batch));
    const FactorWs w = carve_factor(F, batch, ws);
    // F_r c_F: bins of the pairs, inverse length-2N transform, rows n < N;
    // y += [V U_T] ([mu d] . c_rest), inside the inverse column pass where it
    // takes the update, else as a separate pass
    const int rt = (int)(F->r1 + F->r);
    HIPCHK(pack_scale(c, ldc, F->kf, N, batch, w.Zb, rt, F->w, w.dC, st));
    Corr<float> corr;
    const bool fused = rt > 0 && F->ctile && colinv_corr_ok(P->g32, ldy, batch, rt);
    if (fused) {
      corr.U = F->rec();
      corr.ldu = F->ldu;
      corr.r = rt;
      corr.dC = w.dC;
      corr.mode = F->mode;
      corr.ut = F->ctile;
    }
    HIPCHK(dft_bins_inv(w.Zb, F->kf, y, ldy, N, batch, P->g32, P->tb32, w.Z, w.slice, corr, st));
    if (rt > 0 && !fused) HIPCHK(corr_apply_mfma(y, ldy, N, batch, F->rec(), F->ldu, rt, w.dC, st));
    return SLEPIAN_OK;
  });
}

int slepian_project(slepian_plan_t P, const float *x, int64_t ldx, float *y, int64_t ldy, int64_t batch, void *work,
                    size_t work_bytes, void *stream) {
  if (!P) return SLEPIAN_EINVAL;
  return slepian_project_ex(P, P->precision, x, ldx, y, ldy, batch, work, work_bytes, stream);
}

// ---------------------------------------------------------------------------
// The allocation-free projection: its workspace is a file-scope device array
// ---------------------------------------------------------------------------

namespace {
constexpr size_t kNoAllocScratchBytes = (size_t)160 << 20;  // the paper-scale batch in one pass
constexpr int kMaxDevices = 64;
}  // namespace

// Each device that runs the library holds its own copy of this array for the
// life of the process.  In host code `scratch` only names the array: kernels
// get the device address that hipGetSymbolAddress returns for the device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current.
void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) throw Fail{SLEPIAN_ENOTSUP};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    DeviceGuard dg(device);
    void *ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

}  // namespace

int slepian_project_noalloc(slepian_plan_t P, const float *x, int64_t ldx, float *y, int64_t ldy, int64_t batch,
                            void *stream) {
  if (bad_signal_args(P, x, ldx, y, ldy, batch)) return SLEPIAN_EINVAL;
  if (batch == 0) return SLEPIAN_OK;
  if (overlapping(x, ldx, y, ldy, P->N, batch)) return SLEPIAN_EINVAL;
  if (x == y && ldx != ldy) return SLEPIAN_EINVAL;
  // the largest even sub-batch (or the whole batch) whose workspace fits
  auto need = [&](int64_t b) { return op_workspace(P, SLEPIAN_OP_PROJECT, b); };
  int64_t bc = batch;
  if (need(bc) > kNoAllocScratchBytes) {
    int64_t lo = 0, hi = batch / 2;  // in pairs: lo fits (or is 0), hi does not
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) / 2;
      if (need(2 * mid) <= kNoAllocScratchBytes) lo = mid;
      else hi = mid;
    }
    if (lo == 0) return SLEPIAN_ESCRATCH;
    bc = 2 * lo;
  }
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    void *ws = noalloc_scratch(P->device);
    hipStream_t st = (hipStream_t)stream;
    for (int64_t s = 0; s < batch; s += bc) {
      const int64_t n = std::min(bc, batch - s);
      Carver cv(ws);
      ProjWs w = carve_project(P, P->proj, n, cv, P->precision);
      run_fast_op(P, P->proj, 1.0f, 0.0f, x + s * ldx, ldx, y + s * ldy, ldy, n, w, st, P->precision);
    }
    return SLEPIAN_OK;
  });
}

int slepian_apply_b64(slepian_plan_t P, const double *x, int64_t ldx, double *y, int64_t ldy, int64_t batch,
                      void *work, size_t work_bytes, void *stream) {
  if (bad_signal_args(P, x, ldx, y, ldy, batch)) return SLEPIAN_EINVAL;
  if (batch == 0) return SLEPIAN_OK;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    Carver c0(nullptr);
    carve_b64(P, batch, c0);
    void *ws = get_ws(P, work, work_bytes, c0.off + 256);
    Carver cv(ws);
    B64Ws w = carve_b64(P, batch, cv);
    run_b64(P, x, ldx, y, ldy, batch, w, (hipStream_t)stream);
    return SLEPIAN_OK;
  });
}

int slepian_lsq(slepian_plan_t P, int mode, double alpha, const float *y, int64_t ldy, double *x, int64_t ldx,
                int64_t batch, double tol, int max_iter, void *work, size_t work_bytes, void *stream,
                slepian_lsq_report *rep) {
  if (bad_signal_args(P, y, ldy, x, ldx, batch)) return SLEPIAN_EINVAL;
  if (mode != SLEPIAN_PINV && mode != SLEPIAN_TIKHONOV) return SLEPIAN_EINVAL;
  if (max_iter < 0 || !(tol >= 0.0)) return SLEPIAN_EINVAL;
  if (mode == SLEPIAN_TIKHONOV) {
    if (!(alpha > 0.0) || !(P->alpha > 0.0) || std::fabs(alpha - P->alpha) > 1e-12 * P->alpha)
      return SLEPIAN_EINVAL;
  }
  if (rep) std::memset(rep, 0, sizeof(*rep));
  if (batch == 0) return SLEPIAN_OK;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = P->N, b = batch;
    void *ws = get_ws(P, work, work_bytes, op_workspace(P, SLEPIAN_OP_LSQ, b));
    if (mode == SLEPIAN_PINV) {
      static const OpSet none;
      Carver cv(ws);
      PinvWs w = carve_pinv(P, b, cv);
      run_fast_op(P, none, 1.0f, 0.0f, y, ldy, w.t, N, b, w.w, st);
      HIPCHK(cast_f32_to_f64(w.t, N, x, ldx, N, b, st));
      HIPCHK(corr64(y, ldy, x, ldx, N, b, P->U64 + P->pinv.off * N, N, (int)P->pinv.r, P->pinv.d64, w.part, w.dC,
                    st));
      if (rep) {
        rep->converged = 1;
        HIPCHK(hipStreamSynchronize(st));
      }
      return SLEPIAN_OK;
    }
    Carver cv(ws);
    TikWs w = carve_tik(P, b, cv);
    // starting point B y / (1 + alpha) + U5 U5^T y.  As the result itself
    // (max_iter = 0) its correction runs in FP64 (the weights reach
    // 1/(2 sqrt(alpha)) and would amplify FP32 rounding); as the start of the
    // refinement, which removes that rounding, in FP32 on the matrix cores.
    if (max_iter == 0) {
      static const OpSet none;
      run_fast_op(P, none, (float)(1.0 / (1.0 + alpha)), 0.0f, y, ldy, w.x32, N, b, w.pw, st);
      HIPCHK(cast_f32_to_f64(w.x32, N, x, ldx, N, b, st));
      HIPCHK(corr64(y, ldy, x, ldx, N, b, P->U64 + P->tik.off * N, N, (int)P->tik.r, P->tik.d64, w.part64,
                    w.dC64, st));
    } else {
      run_fast_op(P, P->tik, (float)(1.0 / (1.0 + alpha)), 0.0f, y, ldy, w.x32, N, b, w.pw, st);
      HIPCHK(cast_f32_to_f64(w.x32, N, x, ldx, N, b, st));
    }
    if (max_iter == 0 && !rep) return SLEPIAN_OK;
    HIPCHK(cast_f32_to_f64(y, ldy, w.y64, N, N, b, st));
    run_b64(P, w.y64, N, w.By, N, b, w.bw, st);
    HIPCHK(col_norms(w.By, N, N, b, w.nBy, w.npart, st));
    std::vector<double> nBy(b), nr(b);
    HIPCHK(hipMemcpyAsync(nBy.data(), w.nBy, b * sizeof(double), hipMemcpyDeviceToHost, st));
    const float betaM = (float)(1.0 / (1.0 + alpha) - 1.0 / alpha);
    const float gammaM = (float)(1.0 / alpha);
    int it = 0;
    double rel = INFINITY, first = INFINITY;
    bool conv = false;
    // t = B x and u = B^2 x of the current iterate, in FP64: FP64 products for
    // the starting point, then, since B (x + e) = B x + B e, each correction
    // e (FP32 values) adds B e and B (B e) from FP32 products.  Their
    // rounding, about 1e-7 of the correction's size (itself about 1e-7 of
    // x's after the first step), stays far below the residual tolerance.
    run_b64(P, x, ldx, w.t, N, b, w.bw, st);
    run_b64(P, w.t, N, w.u, N, b, w.bw, st);
    for (;; ++it) {
      HIPCHK(lsq_residual_norms(w.By, w.u, x, ldx, alpha, w.rho32, N, b, w.nr, w.npart, st));
      HIPCHK(hipMemcpyAsync(nr.data(), w.nr, b * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      rel = 0.0;
      for (int64_t s = 0; s < b; ++s) {
        // a NaN or Inf in y (or produced from it) shows up in these norms
        if (!std::isfinite(nBy[s]) || !std::isfinite(nr[s])) return SLEPIAN_ENONFINITE;
        const double v = nBy[s] > 0 ? nr[s] / nBy[s] : (nr[s] > 0 ? INFINITY : 0.0);
        rel = std::max(rel, v);
      }
      if (it == 0) first = rel;
      // the tracked residual differs from one recomputed from scratch in
      // FP64 by the FP64 products' rounding (measured near 3e-14 of ||B y||);
      // convergence is claimed only with that margin, so tol <= 1e-12 is
      // never met
      if (rel + kResidualMargin <= tol) {
        conv = true;
        break;
      }
      if (it >= max_iter) break;
      run_fast_op(P, P->tikm, betaM, gammaM, w.rho32, N, w.e32, N, b, w.pw, st);
      HIPCHK(add_f32_to_f64(w.e32, N, x, ldx, N, b, st));
      static const OpSet none;
      run_fast_op(P, none, 1.0f, 0.0f, w.e32, N, w.rho32, N, b, w.pw, st);   // B e
      HIPCHK(add_f32_to_f64(w.rho32, N, w.t, N, N, b, st));
      run_fast_op(P, none, 1.0f, 0.0f, w.rho32, N, w.x32, N, b, w.pw, st);   // B (B e)
      HIPCHK(add_f32_to_f64(w.x32, N, w.u, N, N, b, st));
    }
    if (rep) {
      rep->iterations = it;
      rep->rel_residual = rel;
      rep->rel_residual_first = first;
      rep->converged = conv ? 1 : 0;
    }
    if (max_iter > 0 && !conv) return SLEPIAN_ENOCONV;
    return SLEPIAN_OK;
  });
}

int slepian_coeffs(slepian_plan_t P, const float *x, int64_t ldx, float *c, int64_t ldc, int64_t batch, void *work,
                   size_t work_bytes, void *stream) {
  if (!P || batch < 0) return SLEPIAN_EINVAL;
  if (batch > 0 && (!x || !c || ldx < P->N || ldc < P->K || batch > 32 * 65535)) return SLEPIAN_EINVAL;
  if ((size_t)P->N * (size_t)P->K * sizeof(float) > kCoeffsCap) return SLEPIAN_ENOTSUP;
  if (batch == 0) return SLEPIAN_OK;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = P->N, K = P->K;
    // the vectors' operand image is built on first use and kept by the plan;
    // one call at a time builds or reads it
    std::lock_guard<std::mutex> lock(P->coeffs_mu);
    const int mode = P->precision == SLEPIAN_FP32 ? 0 : 1;
    const int64_t Tn = coeffs_steps(N);
    if (mode == 0 ? !P->SK : !P->SKimg) {
      // all K Slepian vectors, l = 0..K-1 (column l), FP64 then FP32, zero
      // past N; for the BF16 image the FP32 columns are a temporary
      Tridiag T;
      hipStream_t s2 = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
      float *SK = nullptr;
      void *img = nullptr;
      try {
        build_tridiag(P, T, s2);
        const int64_t ldsk = Tn * 32;
        SK = dalloc<float>((size_t)ldsk * K);
        HIPCHK(hipMemsetAsync(SK, 0, (size_t)ldsk * K * sizeof(float), s2));
        DBuf<double> theta(K);
        HIPCHK(tridiag_bisect(T.a, T.e2, N, T.gl, T.gu, T.pivmin, N - K, K, theta.p, s2));
        const size_t per = inviter_scratch_bytes(N, 1) + N * sizeof(double);
        int64_t cv = std::max<int64_t>(1, std::min<int64_t>(K, (int64_t)(inviter_budget() / per)));
        DBuf<char> scratch(inviter_scratch_bytes(N, cv));
        DBuf<double> V((size_t)N * cv);
        for (int64_t j0 = 0; j0 < K; j0 += cv) {
          const int64_t cc = std::min(cv, K - j0);
          // theta[j0 + jj] <-> l = K-1-(j0+jj); normalised column cc-1-jj of V
          HIPCHK(tridiag_inviter(T.a, T.off, N, theta.p + j0, cc, V.p, scratch.p, 3, s2));
          HIPCHK(cast_f64_to_f32(V.p, N, SK + (K - j0 - cc) * ldsk, ldsk, N, cc, s2));
        }
        if (mode == 1) {
          img = dalloc<char>(coeffs_image_bytes(N, K));
          HIPCHK(coeffs_image(1, SK, ldsk, N, K, img, s2));
        }
        HIPCHK(hipStreamSynchronize(s2));
        (void)hipStreamDestroy(s2);
      } catch (...) {
        (void)hipStreamSynchronize(s2);
        (void)hipStreamDestroy(s2);
        dfree(SK);
        dfree(img);
        throw;
      }
      P->ldsk = Tn * 32;
      if (mode == 1) {
        dfree(SK);
        P->SKimg = img;
      } else {
        P->SK = SK;
      }
    }
    const size_t need = op_workspace(P, SLEPIAN_OP_COEFFS, batch);
    void *ws = get_ws(P, work, work_bytes, need);
    Carver cv(ws);
    const int64_t bc = std::min<int64_t>(batch, kCoeffsChunk);
    void *ximg = cv.take<char>(coeffs_image_bytes(N, bc));
    float *part = cv.take<float>(coeffs_part_floats(N, K, bc));
    const void *simg = mode == 0 ? static_cast<const void *>(P->SK) : P->SKimg;
    for (int64_t s0 = 0; s0 < batch; s0 += kCoeffsChunk) {
      const int64_t bb = std::min<int64_t>(kCoeffsChunk, batch - s0);
      HIPCHK(coeffs_image(mode, x + s0 * ldx, ldx, N, bb, ximg, st));
      HIPCHK(coeffs_gemm(mode, simg, ximg, N, K, bb, part, c + s0 * ldc, ldc, st));
    }
    return SLEPIAN_OK;
  });
}

// ---------------------------------------------------------------------------
// Plan files
// ---------------------------------------------------------------------------

namespace {
const char kMagic[8] = {'S', 'L', 'E', 'P', 'P', 'L', 'N', '1'};

struct FileHeader {
  char magic[8];
  int64_t N, K, win_lo, win_hi, u_l0, u_r;
  double W, eps, alpha;
  int32_t precision, pad;
  int64_t proj_off, proj_r, tik_off, tik_r;
  double lam_Km1, lam_K, eps_ach;
};
}  // namespace

int slepian_plan_save(slepian_plan_t P, const char *path) {
  if (!P || !path) return SLEPIAN_EINVAL;
  return guarded([&]() -> int {
    DeviceGuard dg(P->device);
    FileHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kMagic, 8);
    h.N = P->N;
    h.K = P->K;
    h.win_lo = P->win_lo;
    h.win_hi = P->win_hi;
    h.u_l0 = P->u_l0;
    h.u_r = P->u_r;
    h.W = P->W;
    h.eps = P->eps;
    h.alpha = P->alpha;
    h.precision = P->precision;
    h.proj_off = P->proj.off;
    h.proj_r = P->proj.r;
    h.tik_off = P->tik.off;
    h.tik_r = P->tik.r;
    h.lam_Km1 = P->lam_Km1;
    h.lam_K = P->lam_K;
    h.eps_ach = P->eps_ach;
    std::vector<double> U((size_t)P->N * P->u_r);
    if (P->u_r) HIPCHK(hipMemcpy(U.data(), P->U64, U.size() * sizeof(double), hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return SLEPIAN_EIO;
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
    ok = ok && std::fwrite(P->lam.data(), sizeof(double), P->lam.size(), f) == P->lam.size();
    for (const OpSet *o : {&P->proj, &P->pinv, &P->tik, &P->tikm})
      ok = ok && std::fwrite(o->d.data(), sizeof(double), o->d.size(), f) == o->d.size();
    ok = ok && std::fwrite(U.data(), sizeof(double), U.size(), f) == U.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SLEPIAN_OK : SLEPIAN_EIO;
  });
}

int slepian_plan_load(const char *path, int device, slepian_plan_t *out) {
  if (!path || !out) return SLEPIAN_EINVAL;
  *out = nullptr;
  return guarded([&]() -> int {
    // the whole file is read and checked on the host before any device work
    FILE *f = std::fopen(path, "rb");
    if (!f) return SLEPIAN_EIO;
    std::vector<char> buf;
    {
      char chunk[1 << 16];
      size_t got;
      while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) {
        buf.insert(buf.end(), chunk, chunk + got);
        if (buf.size() > ((size_t)1 << 36)) break;  // larger than any valid plan
      }
      std::fclose(f);
    }
    FileHeader h;
    if (buf.size() < sizeof(h)) return SLEPIAN_EIO;
    std::memcpy(&h, buf.data(), sizeof(h));
    if (std::memcmp(h.magic, kMagic, 8) != 0) return SLEPIAN_EIO;
    slepian_plan_opts o{h.alpha, h.K, h.precision, device};
    if (validate_domain(h.N, h.W, h.eps, &o) != SLEPIAN_OK) return SLEPIAN_EIO;
    if (h.win_lo < 0 || h.win_hi < h.win_lo || h.win_hi >= h.N) return SLEPIAN_EIO;
    const int64_t nw = h.win_hi - h.win_lo + 1;
    if (h.u_r < 0 || h.u_r > nw || h.proj_r < 0 || h.tik_r < 0 || h.proj_off < 0 || h.tik_off < 0 ||
        h.proj_off + h.proj_r > h.u_r || h.tik_off + h.tik_r > h.u_r || h.u_l0 < h.win_lo ||
        h.u_l0 + h.u_r > h.win_hi + 1)
      return SLEPIAN_EIO;
    // sizes are bounded by the checks above (N <= 2^21, u_r <= nw <= N), so
    // the expected length is computed without overflow and compared exactly
    const size_t want = sizeof(h) + sizeof(double) * ((size_t)nw + 2 * (size_t)h.proj_r + 2 * (size_t)h.tik_r +
                                                      (size_t)h.N * (size_t)h.u_r);
    if (buf.size() != want) return SLEPIAN_EIO;
    const double *body = reinterpret_cast<const double *>(buf.data() + sizeof(h));
    for (size_t k = 0; k < (want - sizeof(h)) / sizeof(double); ++k)
      if (!std::isfinite(body[k])) return SLEPIAN_EIO;
    int dev = device;
    if (dev < 0) HIPCHK(hipGetDevice(&dev));
    DeviceGuard dg(dev);
    Plan *P = new Plan();
    try {
      P->device = dev;
      P->N = h.N;
      P->K = h.K;
      P->W = h.W;
      P->eps = h.eps;
      P->alpha = h.alpha;
      P->precision = h.precision;
      P->win_lo = h.win_lo;
      P->win_hi = h.win_hi;
      P->u_l0 = h.u_l0;
      P->u_r = h.u_r;
      P->lam_Km1 = h.lam_Km1;
      P->lam_K = h.lam_K;
      P->eps_ach = h.eps_ach;
      const double *q = body;
      P->lam.assign(q, q + nw);
      q += nw;
      P->proj.off = P->pinv.off = h.proj_off;
      P->proj.r = P->pinv.r = h.proj_r;
      P->tik.off = P->tikm.off = h.tik_off;
      P->tik.r = P->tikm.r = h.tik_r;
      for (OpSet *op : {&P->proj, &P->pinv, &P->tik, &P->tikm}) {
        op->d.assign(q, q + op->r);
        q += op->r;
      }
      std::vector<double> U(q, q + (size_t)P->N * P->u_r);
      hipStream_t st = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      try {
        build_fft_state(P, st);
        (void)hipStreamDestroy(st);
      } catch (...) {
        (void)hipStreamDestroy(st);
        throw;
      }
      P->ldu = (P->N + 3) / 4 * 4;
      P->U64 = dalloc<double>((size_t)P->N * std::max<int64_t>(P->u_r, 1));
      P->U32 = dalloc<float>((size_t)P->ldu * std::max<int64_t>(P->u_r, 1));
      if (P->u_r) {
        HIPCHK(hipMemcpy(P->U64, U.data(), U.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(cast_f64_to_f32(P->U64, P->N, P->U32, P->ldu, P->N, P->u_r, nullptr));
        HIPCHK(hipDeviceSynchronize());
      }
      P->tik.set = P->tikm.set = 1;
      for (OpSet *op : {&P->proj, &P->pinv, &P->tik, &P->tikm}) upload_d(*op);
      build_corr_tiles(P, nullptr);
    } catch (...) {
      delete P;
      throw;
    }
    *out = P;
    return SLEPIAN_OK;
  });
}

// ---------------------------------------------------------------------------
// Groups
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

// Plans whose three passes the grouped kernels cover: register-stage rows of
// 8192 points and at most 32 columns.
bool group_three_pass(const Plan *P) {
  const FftGeom &g = P->g32;
  return g.v2 && !g.single() && (g.log2 == 13 || g.log2 == 12) && g.log1 >= 1 && g.log1 <= 5;
}

GroupSpan span_of(const slepian_group_s *G, const slepian_group_s::Span &sp) {
  GroupSpan g;
  g.m = sp.m;
  g.blocks = sp.blocks;
  if (sp.m) {
    g.idx = G->span_buf + sp.off;
    g.start = G->span_buf + sp.off + sp.m;
  }
  return g;
}

void group_partial(const slepian_group_s *G, int var, bool vec, hipStream_t st) {
  const int umode = G->prec == SLEPIAN_MIXED ? 1 : 0;
  HIPCHK(group_corr_partial(umode, 2 - var, vec, G->gp_dev, span_of(G, G->partial[var]), st));
}

void group_colinv_fused(const slepian_group_s *G, int l1, int var, hipStream_t st) {
  const int umode = G->prec == SLEPIAN_MIXED ? 1 : 0;
  HIPCHK(group_colinv_corr(l1, umode, 8 >> var, false, G->gp_dev, span_of(G, G->colinv_corr[l1][var]), st));
  if (l1 == 5)
    HIPCHK(group_colinv_corr(l1, umode, 8 >> var, true, G->gp_dev, span_of(G, G->colinv_corr1[var]), st));
}

// The grouped launches, in the order of the single-plan path: plans whose
// single-pass kernel carries the correction on s2 (independent of the rest),
// everything else on s1.  vec: bit 0 all x, bit 1 all y 16-byte aligned rows.
void launch_grouped(const slepian_group_s *G, hipStream_t s1, hipStream_t s2, int vec) {
  for (int l2 = 9; l2 <= 13; ++l2) HIPCHK(group_single(l2, true, G->gp_dev, span_of(G, G->single_corr[l2]), s2));
  group_partial(G, G->partial_var, vec & 1, s1);
  const int umode = G->prec == SLEPIAN_MIXED ? 1 : 0;
  for (int l1 = 4; l1 <= 5; ++l1) HIPCHK(group_colfwd_corr(l1, umode, G->gp_dev, span_of(G, G->colfwd_corr[l1]), s1));
  HIPCHK(group_corr_reduce(G->gp_dev, span_of(G, G->reduce), s1));
  for (int l2 = 9; l2 <= 13; ++l2) HIPCHK(group_single(l2, false, G->gp_dev, span_of(G, G->single[l2]), s1));
  for (int l1 = 1; l1 <= 5; ++l1) HIPCHK(group_colfwd(l1, G->gp_dev, span_of(G, G->colfwd[l1]), s1));
  HIPCHK(group_row(13, G->gp_dev, span_of(G, G->row[1]), s1));
  HIPCHK(group_row(12, G->gp_dev, span_of(G, G->row[0]), s1));
  for (int l1 = 1; l1 <= 5; ++l1) {
    group_colinv_fused(G, l1, G->colinv_var[l1], s1);
    HIPCHK(group_colinv(l1, G->gp_dev, span_of(G, G->colinv[l1]), s1));
  }
  HIPCHK(group_corr_apply((vec & 2) != 0, G->gp_dev, span_of(G, G->apply), s1));
}

// Autotuning: run the group once (so the intermediates hold this call's
// data), then time each launch that has alternatives, best of two runs per
// alternative, and keep the faster.  The alternatives differ only in how the
// work is cut into workgroups, so every run writes the same results.
// The group's entry in the tuning cache of its first plan that names one:
// "slepian-group-v1 <hash> <plans> <partial> <pass C per L1 = 2..32>", the
// hash (FNV-1a, 64 bits) over each plan's N, W, eps, precision and batch.
uint64_t group_key(const slepian_group_s *G) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  };
  for (size_t i = 0; i < G->plans.size(); ++i) {
    const Plan *P = G->plans[i];
    mix(&P->N, sizeof(P->N));
    mix(&P->W, sizeof(P->W));
    mix(&P->eps, sizeof(P->eps));
    mix(&P->precision, sizeof(P->precision));
    mix(&G->batch[i], sizeof(G->batch[i]));
  }
  return h;
}

const char *group_cache_path(const slepian_group_s *G) {
  for (const Plan *P : G->plans)
    if (!P->tune_cache.empty()) return P->tune_cache.c_str();
  return nullptr;
}

bool group_cache_lookup(slepian_group_s *G) {
  const char *path = group_cache_path(G);
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  const uint64_t key = group_key(G);
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    unsigned long long k = 0;
    long long n = 0;
    int pv = 0, cv[5] = {0, 0, 0, 0, 0};
    if (std::sscanf(line, "slepian-group-v1 %llx %lld %d %d %d %d %d %d", &k, &n, &pv, &cv[0], &cv[1], &cv[2], &cv[3],
                    &cv[4]) != 8)
      continue;
    if (k != key || n != (long long)G->plans.size() || (pv & ~1) != 0) continue;
    bool ok = true;
    for (int v : cv) ok = ok && (v & ~1) == 0;
    if (!ok) continue;
    G->partial_var = pv;
    for (int l1 = 1; l1 <= 5; ++l1) G->colinv_var[l1] = cv[l1 - 1];
    found = true;
  }
  std::fclose(f);
  return found;
}

void group_cache_store(const slepian_group_s *G) {
  const char *path = group_cache_path(G);
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "slepian-group-v1 %016llx %lld %d %d %d %d %d %d\n", (unsigned long long)group_key(G),
               (long long)G->plans.size(), G->partial_var, G->colinv_var[1], G->colinv_var[2], G->colinv_var[3],
               G->colinv_var[4], G->colinv_var[5]);
  std::fclose(f);
}

void tune_group(slepian_group_s *G, hipStream_t st, int vec) {
  if (group_cache_lookup(G)) {
    G->tuned = true;
    G->tuned_from_cache = true;
    return;
  }
  launch_grouped(G, st, st, vec);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    throw Fail{SLEPIAN_EHIP};
  }
  auto timed = [&](auto &&fn) {
    float best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      HIPCHK(hipEventRecord(e0, st));
      fn();
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      best = std::min(best, ms);
    }
    return best;
  };
  try {
    if (G->partial[0].m) {
      const float t0 = timed([&] { group_partial(G, 0, vec & 1, st); });
      const float t1 = timed([&] { group_partial(G, 1, vec & 1, st); });
      G->partial_var = t1 < t0 ? 1 : 0;
    }
    for (int l1 = 1; l1 <= 5; ++l1) {
      if (!G->colinv_corr[l1][0].m && !(l1 == 5 && G->colinv_corr1[0].m)) continue;
      const float t0 = timed([&] { group_colinv_fused(G, l1, 0, st); });
      const float t1 = timed([&] { group_colinv_fused(G, l1, 1, st); });
      G->colinv_var[l1] = t1 < t0 ? 1 : 0;
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  G->tuned = true;
  group_cache_store(G);
}

}  // namespace

extern "C" {

int slepian_group_create(const slepian_plan_t *plans, int n, const int64_t *batch, slepian_group_t *out) {
  if (!plans || !batch || !out || n < 1) return SLEPIAN_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!plans[i] || batch[i] < 0 || batch[i] > 32 * 65535) return SLEPIAN_EINVAL;
    if (plans[i]->device != plans[0]->device) return SLEPIAN_EINVAL;
    if (plans[i]->precision != plans[0]->precision) return SLEPIAN_EINVAL;
    if (plans[i]->precision == SLEPIAN_BF16_RAW) return SLEPIAN_ENOTSUP;
  }
  return guarded([&]() -> int {
    DeviceGuard dg(plans[0]->device);
    slepian_group_s *G = new slepian_group_s();
    try {
      G->device = plans[0]->device;
      G->prec = plans[0]->precision;
      G->plans.assign(plans, plans + n);
      G->batch.assign(batch, batch + n);
      const int umode = G->prec == SLEPIAN_MIXED ? 1 : 0;
      // classify, and lay out the grouped workspace
      G->gp.resize(n);
      size_t wsz = 0;
      auto reserve = [&](size_t bytes) {
        wsz = (wsz + 255) & ~(size_t)255;
        const size_t o = wsz;
        wsz += bytes;
        return o;
      };
      std::vector<size_t> zoff(n, 0), poff(n, 0), doff(n, 0);
      std::vector<char> fused(n, 0);  // single pass with the correction inside
      std::vector<char> fwdc(n, 0);   // pass A forms the coefficients' partials (as a single-plan call does)
      for (int i = 0; i < n; ++i) {
        const Plan *P = plans[i];
        const int64_t b = batch[i];
        if (b == 0) continue;
        const int r = (int)P->proj.r;
        const bool single = P->g32.single() && P->g32.v2;  // register-stage single pass
        if (single && fused_single(P, P->proj, G->prec, b)) {
          G->grouped.push_back(i);
          fused[i] = 1;
          continue;
        }
        if (!single && !group_three_pass(P)) {
          G->other.push_back(i);
          G->ws_other_bytes = std::max(G->ws_other_bytes, op_workspace(P, SLEPIAN_OP_PROJECT, b));
          continue;
        }
        G->grouped.push_back(i);
        if (!single) zoff[i] = reserve((size_t)((b + 1) / 2) * (size_t)P->L * sizeof(cpx<float>));
        fwdc[i] = !single && fwd_corr_applies(P, P->proj, umode, b);
        if (r > 0) {
          const int64_t chunks = fwdc[i] ? colfwd_corr_chunks(P->g32) : corr_nchunks(P->N, b, r);
          poff[i] = reserve((size_t)chunks * corr_rpad(r) * b * sizeof(float));
          doff[i] = reserve((size_t)corr_rpad(r) * b * sizeof(float));
        }
      }
      if (wsz) G->ws = dalloc<char>(wsz + 256);
      if (G->ws_other_bytes) G->ws_other = dalloc<char>(G->ws_other_bytes);
      char *ws = static_cast<char *>(G->ws);
      for (int i : G->grouped) {
        const Plan *P = plans[i];
        GroupPlan &g = G->gp[i];
        g.N = (int)P->N;
        g.b = (int)batch[i];
        g.np = (int)((batch[i] + 1) / 2);
        g.ldx = g.ldy = P->N;
        g.logL = P->g32.logL;
        g.log2 = P->g32.log2;
        g.log1 = P->g32.log1;
        g.chat = P->tb32.chat;
        g.rt1 = P->tb32.row1;
        g.rt2 = P->tb32.row2;
        g.tcol = P->tb32.col;
        g.corr.U = P->U32 + P->proj.off * P->ldu;
        g.corr.ldu = P->ldu;
        g.corr.r = (int)P->proj.r;
        g.corr.d = P->proj.d32;
        if (!fused[i]) {
          const int r = (int)P->proj.r;
          g.corr.mode = umode;
          g.corr.ut = P->ctile[0][umode];
          g.rp = colinv_corr_rp(r, umode);
          g.rpad = corr_rpad(r);
          g.chunks = fwdc[i] ? colfwd_corr_chunks(P->g32) : corr_nchunks(P->N, batch[i], r);
          if (fwdc[i]) g.ftile = P->ftile[0][umode];
          if (!P->g32.single()) g.Z = reinterpret_cast<cpx<float> *>(ws + zoff[i]);
          if (r > 0) {
            g.part = reinterpret_cast<float *>(ws + poff[i]);
            g.corr.dC = reinterpret_cast<float *>(ws + doff[i]);
          }
        }
      }
      // spans
      auto add_span = [&](slepian_group_s::Span &sp, const std::vector<int> &ids, auto &&blocks) {
        std::vector<int> idx, start;
        int64_t tot = 0;
        for (int i : ids) {
          const int64_t nb = blocks(G->gp[i]);
          if (nb <= 0) continue;
          idx.push_back(i);
          start.push_back((int)tot);
          tot += nb;
        }
        if (tot > 0x7fffffff) throw Fail{SLEPIAN_ENOTSUP};
        start.push_back((int)tot);
        sp.m = (int)idx.size();
        sp.blocks = tot;
        sp.off = G->span_host.size();
        G->span_host.insert(G->span_host.end(), idx.begin(), idx.end());
        G->span_host.insert(G->span_host.end(), start.begin(), start.end());
      };
      std::vector<int> by_single_corr[14], by_single[14], mfma, red, by_l1[6], by_l1_fc[6], by_l1_fused[6],
          fused_one, by_l1_plain[6], apply;
      for (int i : G->grouped) {
        const Plan *P = plans[i];
        const int r = (int)P->proj.r;
        if (fused[i]) {
          by_single_corr[P->g32.log2].push_back(i);
          continue;
        }
        if (r > 0 && !fwdc[i]) mfma.push_back(i);
        if (r > 0) red.push_back(i);
        if (P->g32.single()) {
          by_single[P->g32.log2].push_back(i);
          if (r > 0) apply.push_back(i);
          continue;
        }
        (fwdc[i] ? by_l1_fc : by_l1)[P->g32.log1].push_back(i);
        // the update rides on the inverse column pass exactly when the
        // single-plan path fuses it there
        if (r > 0 && colinv_corr_ok(P->g32, P->N, batch[i], r) && P->ctile[0][umode]) {
          (colinv_corr_one(P->g32.log1, G->gp[i].rp) ? fused_one : by_l1_fused[P->g32.log1]).push_back(i);
        } else {
          by_l1_plain[P->g32.log1].push_back(i);
          if (r > 0) apply.push_back(i);
        }
      }
      std::vector<int> three[2];  // rows of 2^12, 2^13 points
      for (int l1 = 1; l1 <= 5; ++l1) {
        for (int i : by_l1[l1]) three[plans[i]->g32.log2 - 12].push_back(i);
        for (int i : by_l1_fc[l1]) three[plans[i]->g32.log2 - 12].push_back(i);
      }
      for (int l2 = 9; l2 <= 13; ++l2) {
        add_span(G->single_corr[l2], by_single_corr[l2], group_blocks_single);
        add_span(G->single[l2], by_single[l2], group_blocks_single);
      }
      for (int v = 0; v < 2; ++v)
        add_span(G->partial[v], mfma, [v](const GroupPlan &g) { return group_blocks_partial(g, 2 - v); });
      add_span(G->reduce, red, group_blocks_reduce);
      for (int l1 = 1; l1 <= 5; ++l1) {
        add_span(G->colfwd[l1], by_l1[l1], group_blocks_colfwd);
        add_span(G->colfwd_corr[l1], by_l1_fc[l1], group_blocks_colfwd_corr);
      }
      for (int k = 0; k < 2; ++k) add_span(G->row[k], three[k], group_blocks_row);
      for (int l1 = 1; l1 <= 5; ++l1) {
        for (int v = 0; v < 2; ++v)
          add_span(G->colinv_corr[l1][v], by_l1_fused[l1],
                   [v](const GroupPlan &g) { return group_blocks_colinv(g, 8 >> v); });
        if (l1 == 5)
          for (int v = 0; v < 2; ++v)
            add_span(G->colinv_corr1[v], fused_one, [v](const GroupPlan &g) { return group_blocks_colinv(g, 8 >> v); });
        add_span(G->colinv[l1], by_l1_plain[l1], group_blocks_colfwd);
      }
      add_span(G->apply, apply, group_blocks_apply);
      G->span_buf = dalloc<int>(G->span_host.size());
      HIPCHK(hipMemcpy(G->span_buf, G->span_host.data(), G->span_host.size() * sizeof(int), hipMemcpyHostToDevice));
      G->gp_dev = dalloc<GroupPlan>(n);
      HIPCHK(hipMemcpy(G->gp_dev, G->gp.data(), n * sizeof(GroupPlan), hipMemcpyHostToDevice));
      HIPCHK(hipStreamCreateWithFlags(&G->cap, hipStreamNonBlocking));
      HIPCHK(hipStreamCreateWithFlags(&G->cap2, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&G->ev_fork, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&G->ev_join, hipEventDisableTiming));
    } catch (...) {
      delete G;
      throw;
    }
    *out = G;
    return SLEPIAN_OK;
  });
}

int slepian_group_project(slepian_group_t G, const float *const *x, float *const *y, void *stream) {
  if (!G || !x || !y) return SLEPIAN_EINVAL;
  const int n = (int)G->plans.size();
  for (int i = 0; i < n; ++i)
    if (G->batch[i] > 0 && (!x[i] || !y[i])) return SLEPIAN_EINVAL;
  return guarded([&]() -> int {
    DeviceGuard dg(G->device);
    hipStream_t st = (hipStream_t)stream;
    bool same = G->lx.size() == (size_t)n;
    for (int i = 0; same && i < n; ++i) same = G->lx[i] == x[i] && G->ly[i] == y[i];
    int vec = 3;
    if (!same) {
      for (int i : G->grouped) {
        G->gp[i].x = x[i];
        G->gp[i].y = y[i];
      }
      // stream-ordered after any earlier launch of this group on `stream`
      HIPCHK(hipMemcpyAsync(G->gp_dev, G->gp.data(), n * sizeof(GroupPlan), hipMemcpyHostToDevice, st));
      G->lx.assign(x, x + n);
      G->ly.assign(y, y + n);
    }
    for (int i : G->grouped) {
      if ((reinterpret_cast<uintptr_t>(x[i]) & 15) != 0 || G->gp[i].ldx % 4 != 0) vec &= ~1;
      if ((reinterpret_cast<uintptr_t>(y[i]) & 15) != 0 || G->gp[i].ldy % 4 != 0) vec &= ~2;
    }
    if (!G->grouped.empty()) {
      if (trace_enabled()) {
        // per-kernel timing needs the launches themselves, not a graph
        launch_grouped(G, st, st, vec);
      } else {
        if (!G->tuned) tune_group(G, st, vec);
        if (!G->exec || G->graph_vec != vec) {
          if (G->exec) (void)hipGraphExecDestroy(G->exec);
          if (G->graph) (void)hipGraphDestroy(G->graph);
          G->exec = nullptr;
          G->graph = nullptr;
          HIPCHK(hipStreamBeginCapture(G->cap, hipStreamCaptureModeThreadLocal));
          try {
            HIPCHK(hipEventRecord(G->ev_fork, G->cap));
            HIPCHK(hipStreamWaitEvent(G->cap2, G->ev_fork, 0));
            launch_grouped(G, G->cap, G->cap2, vec);
            HIPCHK(hipEventRecord(G->ev_join, G->cap2));
            HIPCHK(hipStreamWaitEvent(G->cap, G->ev_join, 0));
          } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(G->cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
          }
          HIPCHK(hipStreamEndCapture(G->cap, &G->graph));
          HIPCHK(hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0));
          G->graph_vec = vec;
        }
        HIPCHK(hipGraphLaunch(G->exec, st));
      }
    }
    for (int i : G->other) {
      const Plan *P = G->plans[i];
      Carver cv(G->ws_other);
      ProjWs w = carve_project(P, P->proj, G->batch[i], cv, G->prec);
      run_fast_op(P, P->proj, 1.0f, 0.0f, x[i], P->N, y[i], P->N, G->batch[i], w, st, G->prec);
    }
    return SLEPIAN_OK;
  });
}

int slepian_group_info(slepian_group_t G, slepian_group_info_t *info) {
  if (!G || !info) return SLEPIAN_EINVAL;
  info->plans = (int32_t)G->plans.size();
  info->grouped = (int32_t)G->grouped.size();
  info->other = (int32_t)G->other.size();
  info->tuned = G->tuned ? (G->tuned_from_cache ? 2 : 1) : 0;
  info->partial_variant = G->partial_var;
  for (int l1 = 1; l1 <= 5; ++l1) info->cic_variant[l1 - 1] = G->colinv_var[l1];
  return SLEPIAN_OK;
}

int slepian_group_destroy(slepian_group_t G) {
  if (!G) return SLEPIAN_OK;
  return guarded([&]() -> int {
    DeviceGuard dg(G->device);
    (void)hipDeviceSynchronize();
    delete G;
    return SLEPIAN_OK;
  });
}

}  // extern "C"

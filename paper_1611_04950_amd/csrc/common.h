// Shared device/host definitions for libslepian (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace slp {

// Complex number with the alignment of a float2/double2 so that LDS and
// global accesses are single 8/16-byte transactions.
template <typename R>
struct alignas(2 * sizeof(R)) cpx {
  R x, y;
};

template <typename R>
__host__ __device__ __forceinline__ cpx<R> mk(R a, R b) { return cpx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R>
__host__ __device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }

// Geometry of the length-L circular convolution used for B x.
//   single pass (log1 == 0): one workgroup holds a whole length-L transform in LDS.
//   three passes: L = L1 * L2, time index n = n2 + L2 * n1, frequency index
//   k = k1 + L1 * k2; pass A does the length-L1 column transforms, pass B the
//   length-L2 row transforms with the spectrum multiply in between, pass C the
//   inverse column transforms.
struct FftGeom {
  int logL = 0;
  int log1 = 0;   // L1 = 2^log1 (0: single pass)
  int log2 = 0;   // L2 = 2^log2
  int logCT = 0;  // columns per pass-A/C workgroup
  int logT = 0;   // length of the sub-transform twiddle table
  int s = 0;      // split of the two-level table for W_L^m: m = (hi << s) | lo
  int v2 = 0;     // 1: register-stage kernels; rows of length R1 R2 R3
  int R1 = 0, R2 = 0, R3 = 0;
  // launch choices of a tuned plan (host side; 0: the process default):
  // cic, the fused inverse column pass's shape (1: one pair per lane and 4
  // wavefronts per workgroup, 2: one pair and 8, 3: two pairs and 4);
  // cicmax, the largest log2 L1 whose inverse column pass takes the update
  int cic = 0, cicmax = 0;
  __host__ __device__ bool single() const { return log1 == 0; }
};

// Per-precision LDS budget: elements of cpx<R> held by one workgroup.
template <typename R> struct Lds;
template <> struct Lds<float> { static constexpr int E = 8192; static constexpr int logE = 13; };
template <> struct Lds<double> { static constexpr int E = 4096; static constexpr int logE = 12; };

constexpr int kThreads = 256;   // threads per FFT workgroup
constexpr int kMaxRankSingle = 256;  // max correction columns handled inside the single-pass kernel

// Device tables of one precision for one FFT geometry.
template <typename R>
struct FftTables {
  const cpx<R> *tw_sub = nullptr;  // W_T^m = exp(-2 pi i m / T), m < T
  const cpx<R> *tw_lo = nullptr;   // W_L^m, m < 2^s
  const cpx<R> *tw_hi = nullptr;   // W_L^(m << s), m < 2^(logL - s)
  const R *chat = nullptr;         // spectrum of B's circulant embedding / L, in pass layout
  const cpx<R> *row1 = nullptr;    // register-stage rows: W_L2^{t k1} stored [k1][t]
  const cpx<R> *row2 = nullptr;    // register-stage rows: W_T^{m k2} stored [k2][m]
  const cpx<R> *col = nullptr;     // register-stage columns: W_L^{k1 n2} stored [k1][n2]
};

// Correction y += U diag(d) U^T x.  U is N x r column-major (ldu).
template <typename R>
struct Corr {
  const R *U = nullptr;
  int64_t ldu = 0;
  int r = 0;
  const R *d = nullptr;      // r weights
  // When set (three-pass path), the inverse column pass also adds U dC, with
  // dC = d (.) U^T x already formed and stored [j][s] (leading dimension b);
  // mode 0: FP32 matrix instructions, 1: BF16 hi/lo.
  const R *dC = nullptr;
  int mode = 0;
  const void *ut = nullptr;  // U's rows laid out for that pass (corr_tile), in `mode`'s number format
};

// One plan's operands for the grouped launches, held in a device table that
// every grouped kernel indexes: signals, FFT tables, correction operands and
// the plan's share of the group workspace (FP32 path).
// The fixed-order chunk sum dC[j b + s] = d[j] sum_c part[(c rpad + j) b + s]
// (blocks workgroups of 32 outputs) as the row pass carries it; ey is set by
// the launch.
struct RowSum {
  const float *part = nullptr;
  const float *d = nullptr;
  float *dC = nullptr;
  int chunks = 0, rpad = 0, b = 0, r = 0, blocks = 0, ey = 0;
};

struct GroupPlan {
  const float *x = nullptr;
  float *y = nullptr;
  int64_t ldx = 0, ldy = 0;
  int N = 0, b = 0, np = 0;  // length, signals, signal pairs
  int logL = 0, log2 = 0, log1 = 0;
  const float *chat = nullptr;
  const cpx<float> *rt1 = nullptr, *rt2 = nullptr, *tcol = nullptr;
  float beta = 1.f, gl = 0.f;
  Corr<float> corr;          // U, ldu, r, d (and dC on the three-pass path)
  const void *ftile = nullptr;  // U laid out for pass A with the coefficients (or null)
  int rp = 0, rpad = 0, chunks = 0;
  cpx<float> *Z = nullptr;   // three-pass intermediate, np * L
  float *part = nullptr;     // correction partials, chunks * rpad * b
};

// A grouped launch covers the workgroups of several plans back to back:
// plans idx[0..m), plan q owning workgroups start[q] .. start[q+1]-1.
struct GroupSpan {
  const int *idx = nullptr;
  const int *start = nullptr;
  int m = 0;
  int64_t blocks = 0;
};

}  // namespace slp

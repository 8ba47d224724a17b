// Register-stage FFT kernels for the product beta * B x + gamma * x.
//
// A row transform of length L2 = R1 R2 R3 runs on T = R2 R3 lanes.  The
// forward transform is decimation in frequency:
//   stage 1: lane t holds x[t + T n1] (n1 < R1), does a length-R1 DFT and
//            multiplies by W_L2^{t k1};
//   stage 2: jobs (k1, m'), m' < R3: length-R2 DFT over t = m' + R3 n2, times
//            W_T^{m' k2};
//   stage 3: jobs (k1, k2): length-R3 DFT over m', giving the spectrum at
//            k = k1 + R1 k2 + R1 R2 k3 in registers.
// The spectrum multiply happens in registers in that (digit-reversed) order,
// with the kernel spectrum stored in the same order, and the inverse runs the
// stages backwards (decimation in time) to natural order.  So each transform
// makes two LDS exchanges and no reordering pass.  The LDS layouts are padded
// (row strides T + 16 and R3 + 1 elements) so that every exchange is free of
// bank conflicts for 8-byte elements.
//
// Column passes of the three-pass product (L = L1 * L2, time index
// n = n2 + L2 n1, frequency index k = k1 + L1 k2) give each lane one column
// n2 and do its length-L1 DFT entirely in registers, with the inter-pass
// twiddle W_L^{n2 k1} applied there, so the row kernel needs none.
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "common.h"
#include "corr_sum.h"
#include "fft_reg.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

template <int R1, int R2, int R3>
struct RowShape {
  static constexpr int L2 = R1 * R2 * R3;
  static constexpr int T = R2 * R3;
  static constexpr int J2 = R1 / R2;
  static constexpr int J3 = R1 / R3;
  static constexpr int S1 = T + 16;
  static constexpr int S2 = R3 + 1;
  static constexpr int S2K = R2 * S2;
  static constexpr int LDS = (R1 * S1 > R1 * S2K) ? R1 * S1 : R1 * S2K;
  static_assert(R1 % R2 == 0 && R1 % R3 == 0, "row radices");
};

// Forward transform, spectrum multiply (spec(z, q) on the R3 values of the
// lane's stage-3 job q, whose spectrum starts at offset (t + T q) R3 of the
// row), inverse transform.  v: lane t's R1 samples x[t + T n1] in, L2 *
// result out.  tw1: the lane's W_L2^{t k1} (k1 < R1); rt2: W_T^{m' k2} in LDS,
// rows k2 of R3 + 1 elements (the padding keeps the stage-3 reads, whose lanes
// differ in k2, free of bank conflicts).
//
// DIR = 1 stops after the spectrum callback (forward transform only; v is
// left undefined); DIR = 2 skips the forward stages and the callback must
// fill all R3 values of each job (inverse transform only; v need not be set).
template <typename R, int R1, int R2, int R3, int DIR = 0, typename Spec>
__device__ __forceinline__ void row_conv_core(cpx<R> (&v)[R1], cpx<R> *S, const cpx<R> (&tw1)[R1],
                                              const cpx<R> *__restrict__ rt2, Spec spec) {
  using RS = RowShape<R1, R2, R3>;
  constexpr int T = RS::T;
  const int t = threadIdx.x;
  cpx<R> w[RS::J2][R2];
  if constexpr (DIR == 2) {
    __syncthreads();  // rt2 staged by the caller
  } else {
  reg::dft<R1, -1>(v);
#pragma unroll
  for (int k1 = 1; k1 < R1; ++k1) v[k1] = cmul(v[k1], tw1[k1]);
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) S[k1 * RS::S1 + t] = v[k1];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RS::J2; ++q) {
    const int g = t + T * q, mp = g % R3, k1 = g / R3;
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) w[q][n2] = S[k1 * RS::S1 + mp + R3 * n2];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RS::J2; ++q) {
    const int g = t + T * q, mp = g % R3, k1 = g / R3;
    reg::dft<R2, -1>(w[q]);
#pragma unroll
    for (int k2 = 1; k2 < R2; ++k2) w[q][k2] = cmul(w[q][k2], rt2[k2 * (R3 + 1) + mp]);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) S[k1 * RS::S2K + k2 * RS::S2 + mp] = w[q][k2];
  }
  __syncthreads();
  }
  cpx<R> z[RS::J3][R3];
#pragma unroll
  for (int q = 0; q < RS::J3; ++q) {
    const int g = t + T * q, k2 = g % R2;
    if constexpr (DIR != 2) {
      const int k1 = g / R2;
#pragma unroll
      for (int m = 0; m < R3; ++m) z[q][m] = S[k1 * RS::S2K + k2 * RS::S2 + m];
      reg::dft<R3, -1>(z[q]);
    }
    spec(z[q], q);
    if constexpr (DIR != 1) {
      reg::dft<R3, +1>(z[q]);
#pragma unroll
      for (int m = 1; m < R3; ++m) z[q][m] = cmulc(z[q][m], rt2[k2 * (R3 + 1) + m]);
    }
  }
  if constexpr (DIR == 1) return;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RS::J3; ++q) {
    const int g = t + T * q, k2 = g % R2, k1 = g / R2;
#pragma unroll
    for (int m = 0; m < R3; ++m) S[k1 * RS::S2K + k2 * RS::S2 + m] = z[q][m];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RS::J2; ++q) {
    const int g = t + T * q, mp = g % R3, k1 = g / R3;
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) w[q][k2] = S[k1 * RS::S2K + k2 * RS::S2 + mp];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RS::J2; ++q) {
    const int g = t + T * q, mp = g % R3, k1 = g / R3;
    reg::dft<R2, +1>(w[q]);
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) S[k1 * RS::S1 + mp + R3 * n2] = w[q][n2];
  }
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) v[k1] = S[k1 * RS::S1 + t];
#pragma unroll
  for (int k1 = 1; k1 < R1; ++k1) v[k1] = cmulc(v[k1], tw1[k1]);
  reg::dft<R1, +1>(v);
}

template <typename R, int R1, int R2, int R3>
__device__ __forceinline__ void load_tw1(cpx<R> (&tw1)[R1], const cpx<R> *__restrict__ rt1) {
  constexpr int T = R2 * R3;
  tw1[0] = cpx<R>{(R)1, (R)0};
#pragma unroll
  for (int k1 = 1; k1 < R1; ++k1) tw1[k1] = rt1[k1 * T + threadIdx.x];
}

// W_T^{m' k2} into LDS rows of R3 + 1 (read after row_conv_core's first
// barrier, so no barrier of its own is needed).
template <typename R, int R1, int R2, int R3>
__device__ __forceinline__ void stage_rt2(cpx<R> *rt2s, const cpx<R> *__restrict__ rt2) {
  constexpr int T = R2 * R3;
  const int t = threadIdx.x;
  rt2s[(t / R3) * (R3 + 1) + t % R3] = rt2[t];
}

// The lane's kernel-spectrum values for its stage-3 jobs, fetched up front so
// their latency overlaps the forward stages: job q covers the R3 contiguous
// values at (t + T q) R3.
template <typename R, int R1, int R2, int R3>
__device__ __forceinline__ void load_spec(R (&chv)[R1 / R3][R3], const R *__restrict__ ch) {
  constexpr int T = R2 * R3;
#pragma unroll
  for (int q = 0; q < R1 / R3; ++q)
#pragma unroll
    for (int k = 0; k < R3; ++k) chv[q][k] = ch[(threadIdx.x + T * q) * R3 + k];
}

// Middle pass of the three-pass product: row k1c of pair pl, in place.
template <typename R, int R1, int R2, int R3>
__device__ __forceinline__ void row_body(cpx<R> *__restrict__ Z, int logL, int log2, const cpx<R> *__restrict__ rt1,
                                         const cpx<R> *__restrict__ rt2, const R *__restrict__ chat, R beta, R gl,
                                         int k1c, int pl) {
  using RS = RowShape<R1, R2, R3>;
  __shared__ cpx<R> S[RS::LDS];
  __shared__ cpx<R> rt2s[R2 * (R3 + 1)];
  cpx<R> *row = Z + ((int64_t)pl << logL) + ((int64_t)k1c << log2);
  const int t = threadIdx.x;
  cpx<R> v[R1];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) v[n1] = row[t + RS::T * n1];
  cpx<R> tw1[R1];
  load_tw1<R, R1, R2, R3>(tw1, rt1);
  R chv[RS::J3][R3];
  load_spec<R, R1, R2, R3>(chv, chat + ((int64_t)k1c << log2));
  stage_rt2<R, R1, R2, R3>(rt2s, rt2);
  row_conv_core<R, R1, R2, R3>(v, S, tw1, rt2s, [&](cpx<R> *z, int q) {
#pragma unroll
    for (int k = 0; k < R3; ++k) z[k] = cscale(z[k], beta * chv[q][k] + gl);
  });
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) row[t + RS::T * n1] = v[n1];
}

template <typename R, int R1, int R2, int R3>
__global__ __launch_bounds__(R2 *R3) void k_row2(cpx<R> *__restrict__ Z, int logL, int log2,
                                                 const cpx<R> *__restrict__ rt1, const cpx<R> *__restrict__ rt2,
                                                 const R *__restrict__ chat, R beta, R gl) {
  row_body<R, R1, R2, R3>(Z, logL, log2, rt1, rt2, chat, beta, gl, blockIdx.x, blockIdx.y);
}

// The row pass with the fixed-order chunk sum of the correction's
// coefficients riding on its first ey rows of workgroups (pass A has written
// the partials; pass C reads dC): the sum takes no launch of its own.
template <int R1, int R2, int R3>
__global__ __launch_bounds__(R2 *R3) void k_row2_sum(cpx<float> *__restrict__ Z, int logL, int log2,
                                                     const cpx<float> *__restrict__ rt1,
                                                     const cpx<float> *__restrict__ rt2,
                                                     const float *__restrict__ chat, float beta, float gl,
                                                     RowSum rs) {
  if ((int)blockIdx.y < rs.ey) {
    __shared__ float red[16][kReduceOuts + 1];
    const int rb = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (rb < rs.blocks)  // uniform per workgroup
      corr_reduce_block<R2 * R3>(rs.part, rs.chunks, rs.rpad, rs.b, rs.r, rs.d, rs.dC, (int64_t)rs.b, 1, rb, red);
    return;
  }
  row_body<float, R1, R2, R3>(Z, logL, log2, rt1, rt2, chat, beta, gl, blockIdx.x, (int)blockIdx.y - rs.ey);
}

// Single-pass product of one signal pair (L = L2).  With CORR the kernel also
// forms C = U^T [x1 x2] (per-lane partial sums, wavefront reductions, a
// fixed-order sum over wavefronts), scales by d, and adds U (d C) to the
// outputs: the whole fast operator of Corollaries 2-4 in one launch.
template <typename R, int R1, int R2, int R3, bool CORR>
__device__ __forceinline__ void single_body(const R *__restrict__ x, int64_t ldx, R *__restrict__ y, int64_t ldy,
                                            int N, int b, const cpx<R> *__restrict__ rt1,
                                            const cpx<R> *__restrict__ rt2, const R *__restrict__ chat, R beta, R gl,
                                            const Corr<R> &corr, int p) {
  using RS = RowShape<R1, R2, R3>;
  constexpr int T = RS::T;
  constexpr int NW = T / 64;
  __shared__ cpx<R> S[RS::LDS];
  __shared__ cpx<R> rt2s[R2 * (R3 + 1)];
  __shared__ R red[CORR ? NW * kMaxRankSingle * 2 : 2];
  __shared__ R dC[CORR ? 2 * kMaxRankSingle : 2];
  const int t = threadIdx.x;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const R *x0 = x + (int64_t)s0 * ldx;
  const R *x1 = x + (int64_t)(has1 ? s1 : s0) * ldx;
  cpx<R> tw1[R1];
  load_tw1<R, R1, R2, R3>(tw1, rt1);
  stage_rt2<R, R1, R2, R3>(rt2s, rt2);
  cpx<R> v[R1];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    const int n = t + T * n1;
    R a = 0, c = 0;
    if (n < N) {
      a = x0[n];
      if (has1) c = x1[n];
    }
    v[n1] = cpx<R>{a, c};
  }
  if constexpr (CORR) {
    const int wave = t >> 6, lane = t & 63;
    for (int j = 0; j < corr.r; ++j) {
      const R *u = corr.U + (int64_t)j * corr.ldu;
      R a0 = 0, a1 = 0;
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) {
        const int n = t + T * n1;
        if (n < N) {
          const R uv = u[n];
          a0 += uv * v[n1].x;
          a1 += uv * v[n1].y;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        a0 += __shfl_xor(a0, off);
        a1 += __shfl_xor(a1, off);
      }
      if (lane == 0) {
        red[(wave * corr.r + j) * 2] = a0;
        red[(wave * corr.r + j) * 2 + 1] = a1;
      }
    }
    __syncthreads();
    for (int j = t; j < corr.r; j += T) {
      R c0 = 0, c1 = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        c0 += red[(w * corr.r + j) * 2];
        c1 += red[(w * corr.r + j) * 2 + 1];
      }
      const R dj = corr.d[j];
      dC[2 * j] = dj * c0;
      dC[2 * j + 1] = dj * c1;
    }
  }
  R chv[RS::J3][R3];
  load_spec<R, R1, R2, R3>(chv, chat);
  row_conv_core<R, R1, R2, R3>(v, S, tw1, rt2s, [&](cpx<R> *z, int q) {
#pragma unroll
    for (int k = 0; k < R3; ++k) z[k] = cscale(z[k], beta * chv[q][k] + gl);
  });
  R *y0 = y + (int64_t)s0 * ldy;
  R *y1 = y + (int64_t)(has1 ? s1 : s0) * ldy;
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    const int n = t + T * n1;
    if (n < N) {
      R a = v[n1].x, c = v[n1].y;
      if constexpr (CORR) {
        for (int j = 0; j < corr.r; ++j) {
          const R uv = corr.U[n + (int64_t)j * corr.ldu];
          a += uv * dC[2 * j];
          c += uv * dC[2 * j + 1];
        }
      }
      y0[n] = a;
      if (has1) y1[n] = c;
    }
  }
}

template <typename R, int R1, int R2, int R3, bool CORR>
__global__ __launch_bounds__(R2 *R3) void k_single2(const R *__restrict__ x, int64_t ldx, R *__restrict__ y,
                                                    int64_t ldy, int N, int b, const cpx<R> *__restrict__ rt1,
                                                    const cpx<R> *__restrict__ rt2, const R *__restrict__ chat,
                                                    R beta, R gl, Corr<R> corr) {
  single_body<R, R1, R2, R3, CORR>(x, ldx, y, ldy, N, b, rt1, rt2, chat, beta, gl, corr, blockIdx.x);
}

// Pass A: lane = column n2 of pair pl; length-L1 DFT of z[n2 + L2 n1] =
// x1 + i x2 (zero for n >= N) in registers, times W_L^{n2 k1}, stored at
// Z[k1][n2].
// EVEN: only the even frequency rows k1 are stored (the length-N DFT bins of
// the fast factorization read no others).
template <typename R, int L1, bool EVEN = false>
__device__ __forceinline__ void colfwd_body(const R *__restrict__ x, int64_t ldx, int N, int b, int pair0, int logL,
                                            int log2, const cpx<R> *__restrict__ tcol, cpx<R> *__restrict__ Z,
                                            int bx, int pl) {
  const int n2 = bx * 256 + threadIdx.x;
  const int p = pair0 + pl;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const R *x0 = x + (int64_t)s0 * ldx;
  const R *x1 = x + (int64_t)(has1 ? s1 : s0) * ldx;
  cpx<R> a[L1];
#pragma unroll
  for (int n1 = 0; n1 < L1; ++n1) {
    const int n = n2 + (n1 << log2);
    R u = 0, v = 0;
    if (n < N) {
      u = x0[n];
      if (has1) v = x1[n];
    }
    a[n1] = cpx<R>{u, v};
  }
  reg::dft<L1, -1>(a);
  cpx<R> *Zp = Z + ((int64_t)pl << logL) + n2;
  Zp[0] = a[0];
#pragma unroll
  for (int k1 = 1; k1 < L1; ++k1)
    if (!EVEN || (k1 & 1) == 0) Zp[(int64_t)k1 << log2] = cmul(a[k1], tcol[(k1 << log2) + n2]);
}

template <typename R, int L1>
__global__ __launch_bounds__(256) void k_colfwd2(const R *__restrict__ x, int64_t ldx, int N, int b, int pair0,
                                                 int logL, int log2, const cpx<R> *__restrict__ tcol,
                                                 cpx<R> *__restrict__ Z) {
  colfwd_body<R, L1>(x, ldx, N, b, pair0, logL, log2, tcol, Z, blockIdx.x, blockIdx.y);
}

template <typename R, int L1>
__global__ __launch_bounds__(256) void k_colfwd2_even(const R *__restrict__ x, int64_t ldx, int N, int b, int pair0,
                                                      int logL, int log2, const cpx<R> *__restrict__ tcol,
                                                      cpx<R> *__restrict__ Z) {
  colfwd_body<R, L1, true>(x, ldx, N, b, pair0, logL, log2, tcol, Z, blockIdx.x, blockIdx.y);
}

// Pass C: lane = column n2 of pair pl; Z[k1][n2] times W_L^{-n2 k1}, inverse
// length-L1 DFT in registers, y1 = Re and y2 = Im for n = n2 + L2 n1 < N
// (only n1 < L1/2 can hold such n because L >= 2N).
// EVEN: the odd frequency rows k1 are known to be zero and are not read.
template <typename R, int L1, bool EVEN = false>
__device__ __forceinline__ void colinv_body(const cpx<R> *__restrict__ Z, int N, int b, int pair0, int logL,
                                            int log2, const cpx<R> *__restrict__ tcol, R *__restrict__ y,
                                            int64_t ldy, int bx, int pl) {
  const int n2 = bx * 256 + threadIdx.x;
  const int p = pair0 + pl;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const cpx<R> *Zp = Z + ((int64_t)pl << logL) + n2;
  cpx<R> a[L1];
  a[0] = Zp[0];
#pragma unroll
  for (int k1 = 1; k1 < L1; ++k1)
    a[k1] = (EVEN && (k1 & 1)) ? cpx<R>{0, 0} : cmulc(Zp[(int64_t)k1 << log2], tcol[(k1 << log2) + n2]);
  reg::dft<L1, +1>(a);
  R *y0 = y + (int64_t)s0 * ldy;
  R *y1 = y + (int64_t)(has1 ? s1 : s0) * ldy;
#pragma unroll
  for (int n1 = 0; n1 < (L1 > 1 ? L1 / 2 : 1); ++n1) {
    const int n = n2 + (n1 << log2);
    if (n < N) {
      y0[n] = a[n1].x;
      if (has1) y1[n] = a[n1].y;
    }
  }
}

template <typename R, int L1>
__global__ __launch_bounds__(256) void k_colinv2(const cpx<R> *__restrict__ Z, int N, int b, int pair0, int logL,
                                                 int log2, const cpx<R> *__restrict__ tcol, R *__restrict__ y,
                                                 int64_t ldy) {
  colinv_body<R, L1>(Z, N, b, pair0, logL, log2, tcol, y, ldy, blockIdx.x, blockIdx.y);
}

template <typename R, int L1>
__global__ __launch_bounds__(256) void k_colinv2_even(const cpx<R> *__restrict__ Z, int N, int b, int pair0,
                                                      int logL, int log2, const cpx<R> *__restrict__ tcol,
                                                      R *__restrict__ y, int64_t ldy) {
  colinv_body<R, L1, true>(Z, N, b, pair0, logL, log2, tcol, y, ldy, blockIdx.x, blockIdx.y);
}

// Column passes for long columns (L1 = A B = 64 .. 512), two stages through
// LDS: with n1 = a + A n1b and k1 = k1b + B k1a, stage 1 is a length-B DFT
// over n1b for each (column, a) times W_L1^{a k1b}, stage 2 a length-A DFT
// over a for each (column, k1b).  A workgroup takes CB adjacent columns of one
// pair; thread (c, a) = (t mod CB, t div CB) owns stage-1 job (c, a) and the
// stage-2 jobs (c, a + A q), q < B / A.  LDS holds [k1b][a][c], so both
// stages touch consecutive columns in consecutive lanes.  Only n1 < L1/2
// carries samples (L >= 2N), so stage 1 reads half of its inputs.
template <typename R, int A, int B, int CB, bool EVEN = false>
__global__ __launch_bounds__(CB *A) void k_colfwd_lds(const R *__restrict__ x, int64_t ldx, int N, int b, int pair0,
                                                      int logL, int log2, const cpx<R> *__restrict__ tcol,
                                                      cpx<R> *__restrict__ Z) {
  constexpr int L1 = A * B, NT = CB * A, J = B / A;
  static_assert(B % A == 0, "column stages");
  __shared__ cpx<R> S[L1 * CB];
  __shared__ cpx<R> tw[L1];  // W_L1^m
  const int t = threadIdx.x, c = t % CB, a = t / CB;
  const int n2 = blockIdx.x * CB + c;
  const int pl = blockIdx.y, p = pair0 + pl;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const R *x0 = x + (int64_t)s0 * ldx;
  const R *x1 = x + (int64_t)(has1 ? s1 : s0) * ldx;
  for (int m = t; m < L1; m += NT) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)L1, &sn, &cs);
    tw[m] = cpx<R>{(R)cs, (R)(-sn)};
  }
  cpx<R> u[B];
#pragma unroll
  for (int n1b = 0; n1b < B; ++n1b) {
    R re = 0, im = 0;
    if (n1b < B / 2) {
      const int n = n2 + ((a + A * n1b) << log2);
      if (n < N) {
        re = x0[n];
        if (has1) im = x1[n];
      }
    }
    u[n1b] = cpx<R>{re, im};
  }
  reg::dft<B, -1>(u);
  __syncthreads();
#pragma unroll
  for (int k1b = 0; k1b < B; ++k1b) S[(k1b * A + a) * CB + c] = k1b ? cmul(u[k1b], tw[a * k1b]) : u[k1b];
  __syncthreads();
  cpx<R> *Zp = Z + ((int64_t)pl << logL) + n2;
#pragma unroll
  for (int q = 0; q < J; ++q) {
    const int k1b = a + A * q;
    cpx<R> v[A];
#pragma unroll
    for (int i = 0; i < A; ++i) v[i] = S[(k1b * A + i) * CB + c];
    reg::dft<A, -1>(v);
#pragma unroll
    for (int k1a = 0; k1a < A; ++k1a) {
      const int k1 = k1b + B * k1a;
      const int64_t o = (int64_t)k1 << log2;
      if (!EVEN || (k1 & 1) == 0) Zp[o] = k1 ? cmul(v[k1a], tcol[o + n2]) : v[k1a];
    }
  }
}

template <typename R, int A, int B, int CB, bool EVEN = false>
__global__ __launch_bounds__(CB *A) void k_colinv_lds(const cpx<R> *__restrict__ Z, int N, int b, int pair0, int logL,
                                                      int log2, const cpx<R> *__restrict__ tcol, R *__restrict__ y,
                                                      int64_t ldy) {
  constexpr int L1 = A * B, NT = CB * A, J = B / A;
  __shared__ cpx<R> S[L1 * CB];
  __shared__ cpx<R> tw[L1];
  const int t = threadIdx.x, c = t % CB, a = t / CB;
  const int n2 = blockIdx.x * CB + c;
  const int pl = blockIdx.y, p = pair0 + pl;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  for (int m = t; m < L1; m += NT) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)L1, &sn, &cs);
    tw[m] = cpx<R>{(R)cs, (R)(-sn)};
  }
  const cpx<R> *Zp = Z + ((int64_t)pl << logL) + n2;
#pragma unroll
  for (int q = 0; q < J; ++q) {
    const int k1b = a + A * q;
    cpx<R> v[A];
#pragma unroll
    for (int k1a = 0; k1a < A; ++k1a) {
      const int k1 = k1b + B * k1a;
      const int64_t o = (int64_t)k1 << log2;
      v[k1a] = (EVEN && (k1 & 1)) ? cpx<R>{0, 0} : k1 ? cmulc(Zp[o], tcol[o + n2]) : Zp[o];
    }
    reg::dft<A, +1>(v);
#pragma unroll
    for (int i = 0; i < A; ++i) S[(k1b * A + i) * CB + c] = v[i];
  }
  __syncthreads();
  cpx<R> u[B];
#pragma unroll
  for (int k1b = 0; k1b < B; ++k1b) {
    const cpx<R> w = S[(k1b * A + a) * CB + c];
    u[k1b] = k1b ? cmulc(w, tw[a * k1b]) : w;
  }
  reg::dft<B, +1>(u);
  R *y0 = y + (int64_t)s0 * ldy;
  R *y1 = y + (int64_t)(has1 ? s1 : s0) * ldy;
#pragma unroll
  for (int n1b = 0; n1b < B / 2; ++n1b) {
    const int n = n2 + ((a + A * n1b) << log2);
    if (n < N) {
      y0[n] = u[n1b].x;
      if (has1) y1[n] = u[n1b].y;
    }
  }
}

// Pass C fused with the correction update y += U dC (Corollary 2's U1 U2^T x
// term).  Each wavefront owns 16 columns c0..c0+15 and 4 PPL signal pairs.
// Lane (col, blk) = (lane % 16, lane / 16) runs the inverse column DFTs of
// PPL pairs and places the surviving rows straight into 16 x 16 matrix-core
// accumulators D[signal slot][column] (row 4 blk + v, column lane % 16), so
// the update U dC runs on the matrix cores over j with no reshuffle: A =
// dC^T (signal slots x j) from memory, B = U^T (j x columns) from U's rows
// laid out for this pass at plan time (build_corr_tile): element (j, n) with
// n = c0 + col + L2 n1 sits at ((cb ROWS + n1) 16 + col) rp + j, so a lane's
// consecutive j are one vector load and a wavefront's loads for one row n1
// are contiguous.  No LDS and no barrier: the wavefronts of a workgroup only
// share the tile through the caches.  With PPL = 1 the slots 4 blk + 2,
// 4 blk + 3 stay zero: half the matrix rows are idle, which costs little and
// halves the registers that hold the DFT inputs.
//   MODE 0: FP32 tile (rp multiple of 16), v_mfma_f32_16x16x4_f32, lane k
//           index blk takes j = 16 g + 4 blk + m in instruction (g, m);
//   MODE 1: BF16 hi and lo planes (rp multiple of 32), three
//           v_mfma_f32_16x16x32_bf16 per 32 j (hi hi, hi lo, lo hi).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Loads and stores at a wavefront-uniform base plus a 32-bit byte offset per
// lane (the base stays in scalar registers, the lane keeps one 32-bit
// offset instead of a 64-bit address).
template <typename T>
__device__ __forceinline__ T ld_at(const T *base, uint32_t byte_off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_at(T *base, uint32_t byte_off, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off) = v;
}

// Waves per SIMD the fused pass is compiled for (caps its registers; L1 = 32
// keeps 64 complex inputs per lane and is compiled for 3).
constexpr int kCicWaves = 6;

template <int L1, int MODE, int CW, int PPL, bool EVEN = false, bool ONE = false>
__device__ __forceinline__ void colinv_corr_body(const cpx<float> *__restrict__ Z, int N, int b, int pair0, int np,
                                                 int logL, int log2, const cpx<float> *__restrict__ tcol,
                                                 float *__restrict__ y, int64_t ldy, const void *__restrict__ ut,
                                                 int r, int rp, const float *__restrict__ dC, int cb, int by) {
  constexpr int ROWS = L1 > 1 ? L1 / 2 : 1;
  static_assert(PPL == 1 || PPL == 2, "pairs per lane");
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, blk = lane >> 4;
  const int pw = (by * CW + wave) * 4 * PPL;  // first pair of the wavefront, within the slice
  // LDSU (BF16 planes, one-step contraction, L1 = 32): the column block's U
  // tile (hi and lo planes, 16 rows of 1 KB each) is staged once per
  // workgroup in LDS by direct-to-LDS loads, instead of every wavefront
  // reading it through the caches.  In LDS the 16-byte piece blk of column
  // col in a row sits at slot blk ^ ((col / 4) % 4), so that the 16 lanes of
  // one read (16 columns) hit 16 different bank groups; the lane that fills
  // a slot fetches the piece that belongs there.  Every wavefront then takes
  // part in one barrier, so a wavefront past the pairs runs the pass on pair
  // 0's values and stores nothing.
  constexpr bool LDSU = MODE == 1 && ONE;
  static_assert(!LDSU || L1 == 32, "staged tile: 16 rows of 16 columns x 32 j");
  __shared__ __align__(16) char utl[LDSU ? 2 * 16 * 1024 : 16];
  if constexpr (LDSU) {
    if (by * CW * 4 * PPL >= np) return;  // the whole workgroup is past the pairs (uniform)
    const char *th = static_cast<const char *>(ut) + (int64_t)cb * (16 * 1024);
    const char *tlo = th + (((int64_t)ROWS << log2) * 32) * 2;
    const int cq = lane >> 2, sl = lane & 3;
    const uint32_t src = (uint32_t)cq * 64u + (uint32_t)(sl ^ ((cq >> 2) & 3)) * 16u;
    for (int k = wave; k < 32; k += CW)
      __builtin_amdgcn_global_load_lds((k < 16 ? th : tlo) + (k & 15) * 1024 + src,
                                       (__attribute__((address_space(3))) void *)(utl + k * 1024), 16, 0, 0);
  } else {
    if (pw >= np) return;  // uniform per wavefront; the kernel has no barrier
  }
  const int pwz = pw < np ? pw : 0;  // LDSU: a wavefront past the pairs reads pair 0
  const int c0 = cb * 16, n2 = c0 + col;
  // lane offsets below stay under 2^32 bytes: pairs pw .. pw + 4 PPL - 1
  // span 4 PPL L complex values; the host bounds ldy, r and b
  const cpx<float> *Zw = Z + ((int64_t)pwz << logL) + c0;
  cpx<float> a[PPL][L1];
#pragma unroll
  for (int h = 0; h < PPL; ++h) {
    const int q = pw + PPL * blk + h < np ? PPL * blk + h : 0;
    const uint32_t zo = (((uint32_t)q << logL) + (uint32_t)col) * 8u;
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1)
      a[h][k1] = (EVEN && (k1 & 1)) ? cpx<float>{0.f, 0.f} : ld_at(Zw, zo + ((uint32_t)k1 << (log2 + 3)));
  }
  // W_L^{k1 n2} = W_L^{(k1 mod 8) n2} W_L^{8 (k1 div 8) n2}: eight plus L1/8
  // table loads per lane instead of L1, one extra rounding per factor.
  constexpr int TH = L1 > 8 ? L1 / 8 : 1;
  const cpx<float> *tc = tcol + c0;
  cpx<float> tl[L1 < 8 ? L1 : 8], th[TH];
#pragma unroll
  for (int k = 1; k < (L1 < 8 ? L1 : 8); ++k) tl[k] = ld_at(tc, (((uint32_t)k << log2) + (uint32_t)col) * 8u);
#pragma unroll
  for (int m = 1; m < TH; ++m) th[m] = ld_at(tc, (((uint32_t)(8 * m) << log2) + (uint32_t)col) * 8u);
#pragma unroll
  for (int h = 0; h < PPL; ++h) {
#pragma unroll
    for (int k1 = 1; k1 < L1; ++k1) {
      const int kl = k1 & 7, kh = k1 >> 3;
      const cpx<float> w = kh == 0 ? tl[kl] : (kl == 0 ? th[kh] : cmul(tl[kl], th[kh]));
      a[h][k1] = cmulc(a[h][k1], w);
    }
    reg::dft<L1, +1>(a[h]);
  }
  // A row i = lane % 16 is signal slot i: slot 4 q + v holds signal
  // 2 (pair0 + pw + PPL q) + v (PPL = 2), or 2 (pair0 + pw + q) + v for v < 2
  // and nothing for v >= 2 (PPL = 1).
  const int iq = (lane & 15) >> 2, iv = lane & 3;
  const int ipl = pw + PPL * iq + (iv >> 1);
  const int sa = 2 * (pair0 + ipl) + (iv & 1);
  const bool sav = (PPL == 2 || iv < 2) && ipl < np && sa < b;
  const uint32_t sac = sav ? (uint32_t)sa : 0u;
  const uint32_t tile_row = 16u * (uint32_t)rp;  // elements per row n1 of one column block
  float *yw = y + (int64_t)2 * (pair0 + pw) * ldy;
  // ONE (the host launches it for rp = 32, rank <= 32): the contraction over
  // j is one step per row, the A operand is the same for every row and is
  // formed once, and a chunk's tile loads are all in flight together.  Lane
  // (col, blk) holds dC^T[col][j] for j = 8 blk + e (MODE 1) or
  // j = 16 g + 4 blk + m (MODE 0, g = e / 4, m = e % 4).  The sums run in the
  // same order as the general loop's, so both give the same bits.
  constexpr bool one = ONE;
  float dcv[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int j = MODE ? 8 * blk + e : 16 * (e >> 2) + 4 * blk + (e & 3);
    dcv[e] = (one && sav && j < r) ? ld_at(dC, ((uint32_t)j * (uint32_t)b + sac) * 4u) : 0.f;
  }
  bf16x8 ahi1, alo1;
  if constexpr (MODE == 1 && one) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const __bf16 hh = (__bf16)dcv[e];
      ahi1[e] = hh;
      alo1[e] = (__bf16)(dcv[e] - (float)hh);
    }
  }
  if constexpr (LDSU) {
    // this wavefront's tile loads have landed; the barrier makes all visible
    __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));  // vmcnt(0)
    __syncthreads();
  }
  // every row of this column block lies below N: stores need only the
  // signal check (uniform per wavefront)
  const bool full = c0 + 15 + ((ROWS - 1) << log2) < N;
  // Rows go through the matrix cores in chunks of at most eight, so only one
  // chunk's accumulators are live next to the DFT outputs.
  constexpr int RC = ROWS < 8 ? ROWS : 8;
#pragma unroll
  for (int rc = 0; rc < ROWS; rc += RC) {
    f32x4 acc[RC];
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int h = 0; h < PPL; ++h) {
        const bool live = pw + PPL * blk + h < np;
        acc[i][2 * h] = live ? a[h][rc + i].x : 0.f;
        acc[i][2 * h + 1] = live ? a[h][rc + i].y : 0.f;
      }
    }
    const int64_t base = ((int64_t)cb * ROWS + rc) * tile_row;
    if constexpr (MODE == 0) {
      const float *T = static_cast<const float *>(ut) + base;
      const uint32_t lo = (uint32_t)col * rp + 4u * blk;
      if constexpr (one) {
        float4 u0[RC], u1[RC];
#pragma unroll
        for (int i = 0; i < RC; ++i) {
          u0[i] = ld_at(reinterpret_cast<const float4 *>(T), (lo + i * tile_row) * 4u);
          u1[i] = ld_at(reinterpret_cast<const float4 *>(T), (lo + i * tile_row + 16u) * 4u);
        }
#pragma unroll
        for (int i = 0; i < RC; ++i) {
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(dcv[0], u0[i].x, acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(dcv[1], u0[i].y, acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(dcv[2], u0[i].z, acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(dcv[3], u0[i].w, acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(dcv[4], u1[i].x, acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(dcv[5], u1[i].y, acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(dcv[6], u1[i].z, acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(dcv[7], u1[i].w, acc[i], 0, 0, 0);
        }
      } else {
        for (int g = 0; g < rp; g += 16) {
          float av[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int j = g + 4 * blk + m;
            av[m] = (sav && j < r) ? ld_at(dC, ((uint32_t)j * (uint32_t)b + sac) * 4u) : 0.f;
          }
#pragma unroll
          for (int i = 0; i < RC; ++i) {
            const float4 u = ld_at(reinterpret_cast<const float4 *>(T), (lo + i * tile_row + g) * 4u);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0], u.x, acc[i], 0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1], u.y, acc[i], 0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2], u.z, acc[i], 0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[3], u.w, acc[i], 0, 0, 0);
          }
        }
      }
    } else {
      const int64_t plane = ((int64_t)ROWS << log2) * rp;
      const __bf16 *Th = static_cast<const __bf16 *>(ut) + base;
      const __bf16 *Tl = Th + plane;
      const uint32_t lo = (uint32_t)col * rp + 8u * blk;
      if constexpr (one) {
        bf16x8 bhi[RC], blo[RC];
        if constexpr (LDSU) {
          const int so = col * 64 + ((blk ^ ((col >> 2) & 3)) << 4);
#pragma unroll
          for (int i = 0; i < RC; ++i) {
            bhi[i] = *reinterpret_cast<const bf16x8 *>(utl + (rc + i) * 1024 + so);
            blo[i] = *reinterpret_cast<const bf16x8 *>(utl + (16 + rc + i) * 1024 + so);
          }
        } else {
#pragma unroll
          for (int i = 0; i < RC; ++i) {
            const uint32_t o = (lo + i * tile_row) * 2u;
            bhi[i] = ld_at(reinterpret_cast<const bf16x8 *>(Th), o);
            blo[i] = ld_at(reinterpret_cast<const bf16x8 *>(Tl), o);
          }
        }
#pragma unroll
        for (int i = 0; i < RC; ++i) {
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi1, bhi[i], acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi1, blo[i], acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo1, bhi[i], acc[i], 0, 0, 0);
        }
      } else {
        for (int g = 0; g < rp; g += 32) {
          bf16x8 ahi, alo;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int j = g + 8 * blk + e;
            const float av = (sav && j < r) ? ld_at(dC, ((uint32_t)j * (uint32_t)b + sac) * 4u) : 0.f;
            const __bf16 hh = (__bf16)av;
            ahi[e] = hh;
            alo[e] = (__bf16)(av - (float)hh);
          }
#pragma unroll
          for (int i = 0; i < RC; ++i) {
            const uint32_t o = (lo + i * tile_row + g) * 2u;
            const bf16x8 bhi = ld_at(reinterpret_cast<const bf16x8 *>(Th), o);
            const bf16x8 blo = ld_at(reinterpret_cast<const bf16x8 *>(Tl), o);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[i], 0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[i], 0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[i], 0, 0, 0);
          }
        }
      }
    }
    // D[4 blk + v][col] -> signal slot 4 blk + v at n = n2 + L2 (rc + i)
#pragma unroll
    for (int v = 0; v < 2 * PPL; ++v) {
      const int pl = pw + PPL * blk + (v >> 1);
      const int sg = 2 * (pair0 + pl) + (v & 1);
      if (pl >= np || sg >= b) continue;
      const uint32_t so = (uint32_t)(2 * PPL * blk + v) * (uint32_t)ldy + (uint32_t)n2;
      if (full) {
#pragma unroll
        for (int i = 0; i < RC; ++i) st_at(yw, (so + ((uint32_t)(rc + i) << log2)) * 4u, acc[i][v]);
      } else {
#pragma unroll
        for (int i = 0; i < RC; ++i) {
          const int n = n2 + ((rc + i) << log2);
          if (n < N) st_at(yw, (so + ((uint32_t)(rc + i) << log2)) * 4u, acc[i][v]);
        }
      }
    }
  }
}

template <int L1, int MODE, int CW, int PPL, bool EVEN = false, bool ONE = false>
__global__ __launch_bounds__(64 * CW, L1 >= 32 ? 3 : kCicWaves) void k_colinv_corr(const cpx<float> *__restrict__ Z, int N, int b, int pair0,
                                                         int np, int logL, int log2,
                                                         const cpx<float> *__restrict__ tcol, float *__restrict__ y,
                                                         int64_t ldy, const void *__restrict__ ut, int r, int rp,
                                                         const float *__restrict__ dC) {
  // Workgroups are dealt to the eight XCDs round-robin by linear id; give
  // each XCD a contiguous run of column blocks, so the two 64-byte halves of
  // a 128-byte line of y are handled within one L2.
  const int gx = gridDim.x;
  const int cb = (gx & 7) ? (int)blockIdx.x : (int)(blockIdx.x & 7) * (gx >> 3) + (int)(blockIdx.x >> 3);
  colinv_corr_body<L1, MODE, CW, PPL, EVEN, ONE>(Z, N, b, pair0, np, logL, log2, tcol, y, ldy, ut, r, rp, dC, cb,
                                                 blockIdx.y);
}

// U's rows in the order the fused inverse column pass reads them (see
// colinv_corr_body): FP32 (mode 0), or BF16 hi and lo planes (mode 1, lo =
// the rounding error of hi), zero for n >= N and j >= r.
__global__ void k_corr_tile(const float *__restrict__ U, int64_t ldu, int N, int r, int log2, int rows, int rp,
                            int mode, void *__restrict__ out) {
  const int64_t total = ((int64_t)rows << log2) * rp;  // elements per plane
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % rp);
    const int64_t q = e / rp;
    const int c = (int)(q & 15);
    const int64_t q2 = q >> 4;
    const int n1 = (int)(q2 % rows);
    const int64_t cb = q2 / rows;
    const int64_t n = cb * 16 + c + ((int64_t)n1 << log2);
    const float u = (j < r && n < N) ? U[(int64_t)j * ldu + n] : 0.f;
    if (mode == 0) {
      static_cast<float *>(out)[e] = u;
    } else {
      const __bf16 h = (__bf16)u;
      static_cast<__bf16 *>(out)[e] = h;
      static_cast<__bf16 *>(out)[total + e] = (__bf16)(u - (float)h);
    }
  }
}

size_t corr_tile_bytes(int log1, int log2, int r, int mode) {
  const int64_t rows = log1 > 0 ? ((int64_t)1 << log1) / 2 : 1;
  const int64_t e = (rows << log2) * colinv_corr_rp(r, mode);
  return mode == 0 ? (size_t)e * sizeof(float) : (size_t)e * 2 * sizeof(__bf16);
}

hipError_t build_corr_tile(const float *U, int64_t ldu, int N, int r, int log1, int log2, int mode, void *out,
                           hipStream_t st) {
  const int rows = log1 > 0 ? (1 << log1) / 2 : 1;
  const int64_t total = ((int64_t)rows << log2) * colinv_corr_rp(r, mode);
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  SLP_LAUNCH("corr_tile", k_corr_tile, dim3((unsigned)blocks), dim3(256), 0, st, U, ldu, N, r, log2, rows,
             colinv_corr_rp(r, mode), mode, out);
  return hipGetLastError();
}

// ---- pass A fused with the correction's coefficients ----
//
// Pass A also forms the chunk partials of C = U^T X (Corollary 2's U^T x)
// from the signal values it loads, so x is read from memory once for both.
// A workgroup owns 16 columns c0..c0+15 and 16 signal pairs (4 per
// wavefront); lane (col, blk) = (lane % 16, lane / 16) loads rows n1 < R =
// L1/2 (the rows that can hold n < N, as L >= 2N) of column c0 + col for its
// wavefront's pair blk, keeps them for its column DFT and stores them in LDS
// as sample q = col R + n1 of xs[wave][slot 2 blk + c] (at col CS + n1, CS =
// R + 4: padded against bank conflicts).  After one barrier the column
// block's partial sum over its 16 R samples runs on the matrix cores for all
// 32 signals of the workgroup, the T = Q / 32 steps dealt evenly to the four
// wavefronts: step t takes samples q = 32 t + 8 g + e (e < 8, g = lane / 16);
// the A operand (U^T, 16 j at a time) comes from the column block's tile
// (k_fwd_tile, built with the plan), lane (m, g) holding U[n_q][16 jt + m];
// the B operand (16 signals at a time, sb = 0, 1) comes from LDS, lane (s, g)
// holding x[n_q] of signal 16 sb + s of the workgroup.
//   MODE 0: FP32, v_mfma_f32_16x16x4_f32, instruction e takes sample q(e, g)
//           from lane group g;
//   MODE 1: BF16 hi and lo planes, three v_mfma_f32_16x16x32_bf16 per step
//           (hi hi, hi lo, lo hi), FP32 accumulation.
// The wavefronts' sums meet in LDS (reusing xs), are added in a fixed order,
// and one partial per (column block, signal) reaches memory, at
// part[(cb rpad + j) b + s]: the layout the fixed-order chunk sum reads, with
// the column blocks as its chunks.
constexpr int kFcWaves = 4;

template <int L1, int MODE>
__device__ __forceinline__ void colfwd_corr_body(const float *__restrict__ x, int64_t ldx, int N, int b, int np,
                                                 int logL, int log2, const cpx<float> *__restrict__ tcol,
                                                 cpx<float> *__restrict__ Z, const void *__restrict__ ft, int r,
                                                 float *__restrict__ part, int rpad, int cb, int by) {
  constexpr int R = L1 / 2;  // rows n1 that can hold n < N
  constexpr int Q = 16 * R;  // samples of one signal in the column block
  constexpr int T = Q / 32;  // matrix steps
  constexpr int TW = T / kFcWaves;  // steps per wavefront
  // LDS strides padded by 16 bytes: a column's R samples at stride CS, a
  // slot (signal) at stride SS, so that the 16 lanes of a store (16 columns)
  // and of an operand read (16 signals) each hit 16 different bank groups
  constexpr int CS = R + 4, SS = 16 * CS + 4;
  static_assert(R >= 8 && T % kFcWaves == 0, "column length");
  // the wavefronts' sums (2 x 2 tiles of 4 x 64 values each) fit in xs
  static_assert(kFcWaves * 8 * SS >= kFcWaves * 4 * 4 * 64, "reduction space");
  __shared__ __align__(16) float xs[kFcWaves][8][SS];
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, blk = lane >> 4;
  const int pg = by * 4 * kFcWaves;      // first pair of the workgroup
  const int pw = pg + wave * 4;          // first pair of the wavefront
  const int n2 = cb * 16 + col;
  const int p = pw + blk;
  const bool pv = p < np;
  const bool has1 = pv && 2 * p + 1 < b;
  const float *x0 = x + (int64_t)(pv ? 2 * p : 0) * ldx;
  const float *x1 = x + (int64_t)(has1 ? 2 * p + 1 : 0) * ldx;
  cpx<float> a[L1];
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) {
    const int n = n2 + (n1 << log2);
    a[n1].x = (pv && n < N) ? x0[n] : 0.f;
    a[n1].y = (has1 && n < N) ? x1[n] : 0.f;
  }
#pragma unroll
  for (int n1 = R; n1 < L1; ++n1) a[n1] = cpx<float>{0.f, 0.f};
  // The column's twiddles, loaded with the samples so that no load sits
  // between the stores of Z below: W_L^{k1 n2} = W_L^{(k1 mod 8) n2}
  // W_L^{8 (k1 div 8) n2}, seven plus L1/8 - 1 table entries per lane.
  constexpr int TH = L1 / 8;
  const cpx<float> *tc = tcol + n2;
  cpx<float> tl[8], th[TH];
#pragma unroll
  for (int k = 1; k < 8; ++k) tl[k] = tc[k << log2];
#pragma unroll
  for (int m = 1; m < TH; ++m) th[m] = tc[(8 * m) << log2];
  const int s = lane & 15, g = lane >> 4;
  const int njt = (r + 15) >> 4;  // 16-column tiles of U (1 or 2)
  // the wavefront's A operands, loaded with the samples too, so that the
  // matrix phase waits on no memory operation issued after the stores of Z:
  // per step and U tile, two 16-byte pieces (FP32 samples e < 4 and e >= 4,
  // or the BF16 hi and lo planes)
  float4 ua[TW][2][2];
#pragma unroll
  for (int tt = 0; tt < TW; ++tt)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int64_t tile = ((int64_t)cb * T + wave * TW + tt) * njt + (jt < njt ? jt : 0);
      const float4 *Tj = reinterpret_cast<const float4 *>(static_cast<const char *>(ft) + tile * 2048);
      ua[tt][jt][0] = Tj[lane];
      ua[tt][jt][1] = Tj[64 + lane];
    }
  float *xw0 = &xs[wave][2 * blk][col * CS];
  float *xw1 = &xs[wave][2 * blk + 1][col * CS];
#pragma unroll
  for (int n1 = 0; n1 < R; n1 += 4) {
    *reinterpret_cast<float4 *>(xw0 + n1) = float4{a[n1].x, a[n1 + 1].x, a[n1 + 2].x, a[n1 + 3].x};
    *reinterpret_cast<float4 *>(xw1 + n1) = float4{a[n1].y, a[n1 + 1].y, a[n1 + 2].y, a[n1 + 3].y};
  }
  reg::dft<L1, -1>(a);
  // every load of the lane (samples, twiddles, A operands) has landed before
  // the first store of Z, so the matrix phase below waits on none of the
  // stores (vector memory operations complete in order)
  __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));  // vmcnt(0)
  if (pv) {
    cpx<float> *Zp = Z + ((int64_t)p << logL) + n2;
    Zp[0] = a[0];
#pragma unroll
    for (int k1 = 1; k1 < L1; ++k1) {
      const int kl = k1 & 7, kh = k1 >> 3;
      const cpx<float> w = kh == 0 ? tl[kl] : (kl == 0 ? th[kh] : cmul(tl[kl], th[kh]));
      Zp[(int64_t)k1 << log2] = cmul(a[k1], w);
    }
  }
  __syncthreads();
  f32x4 acc[2][2];
#pragma unroll
  for (int jt = 0; jt < 2; ++jt)
#pragma unroll
    for (int sb = 0; sb < 2; ++sb) acc[jt][sb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) {
    const int t = wave * TW + tt;
    float bv[2][8];
#pragma unroll
    for (int sb = 0; sb < 2; ++sb) {
      // signal 16 sb + s of the workgroup: wavefront 2 sb + s / 8, slot s % 8;
      // samples q = 32 t + 8 g + e, i.e. column q / R, rows q % R .. + 7
      const int q0 = 32 * t + 8 * g;
      const float *xr = &xs[2 * sb + (s >> 3)][s & 7][(q0 / R) * CS + q0 % R];
      const float4 v0 = *reinterpret_cast<const float4 *>(xr);
      const float4 v1 = *reinterpret_cast<const float4 *>(xr + 4);
      bv[sb][0] = v0.x; bv[sb][1] = v0.y; bv[sb][2] = v0.z; bv[sb][3] = v0.w;
      bv[sb][4] = v1.x; bv[sb][5] = v1.y; bv[sb][6] = v1.z; bv[sb][7] = v1.w;
    }
    if constexpr (MODE == 0) {
#pragma unroll
      for (int jt = 0; jt < 2; ++jt) {
        if (jt >= njt) break;
        const float4 u0 = ua[tt][jt][0], u1 = ua[tt][jt][1];
        const float uv[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
        for (int sb = 0; sb < 2; ++sb)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            acc[jt][sb] = __builtin_amdgcn_mfma_f32_16x16x4f32(uv[e], bv[sb][e], acc[jt][sb], 0, 0, 0);
      }
    } else {
      bf16x8 bhi[2], blo[2];
#pragma unroll
      for (int sb = 0; sb < 2; ++sb)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const __bf16 h = (__bf16)bv[sb][e];
          bhi[sb][e] = h;
          blo[sb][e] = (__bf16)(bv[sb][e] - (float)h);
        }
#pragma unroll
      for (int jt = 0; jt < 2; ++jt) {
        if (jt >= njt) break;
        const bf16x8 ahi = __builtin_bit_cast(bf16x8, ua[tt][jt][0]);
        const bf16x8 alo = __builtin_bit_cast(bf16x8, ua[tt][jt][1]);
#pragma unroll
        for (int sb = 0; sb < 2; ++sb) {
          acc[jt][sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi[sb], acc[jt][sb], 0, 0, 0);
          acc[jt][sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo[sb], acc[jt][sb], 0, 0, 0);
          acc[jt][sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi[sb], acc[jt][sb], 0, 0, 0);
        }
      }
    }
  }
  // the four wavefronts' sums, red[wave][jt][sb][lane][v], added in wave order
  __syncthreads();  // every wavefront is done reading xs
  float *red = &xs[0][0][0];
  static_assert(sizeof(xs) >= 4 * 2 * 2 * 64 * 4 * sizeof(float), "reduction space");
#pragma unroll
  for (int jt = 0; jt < 2; ++jt)
#pragma unroll
    for (int sb = 0; sb < 2; ++sb)
      *reinterpret_cast<f32x4 *>(red + (((wave * 2 + jt) * 2 + sb) * 64 + lane) * 4) = acc[jt][sb];
  __syncthreads();
  // thread (jt, sb, l) = (tid / 128, tid / 64 % 2, tid % 64): D[4 g + v][s]
  // of tile (jt, sb), i.e. U column 16 jt + 4 (l / 16) + v, signal 16 sb + l % 16
  const int tid = threadIdx.x;
  const int l = tid & 63, sb = (tid >> 6) & 1, jt = tid >> 7;
  f32x4 t4 = *reinterpret_cast<const f32x4 *>(red + (((0 * 2 + jt) * 2 + sb) * 64 + l) * 4);
#pragma unroll
  for (int w = 1; w < kFcWaves; ++w) t4 += *reinterpret_cast<const f32x4 *>(red + (((w * 2 + jt) * 2 + sb) * 64 + l) * 4);
  const int sg = 2 * pg + 16 * sb + (l & 15);
  if (jt < njt && sg < b) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = 16 * jt + 4 * (l >> 4) + v;
      if (j < r) part[((int64_t)cb * rpad + j) * b + sg] = t4[v];
    }
  }
}

template <int L1, int MODE>
__global__ __launch_bounds__(64 * kFcWaves, 3) void k_colfwd_corr(const float *__restrict__ x, int64_t ldx, int N, int b,
                                                               int np, int logL, int log2,
                                                               const cpx<float> *__restrict__ tcol,
                                                               cpx<float> *__restrict__ Z,
                                                               const void *__restrict__ ft, int r,
                                                               float *__restrict__ part, int rpad) {
  // each XCD takes a contiguous run of column blocks, so the two 64-byte
  // halves of a 128-byte line of x are read within one L2
  const int gx = gridDim.x;
  const int cb = (gx & 7) ? (int)blockIdx.x : (int)(blockIdx.x & 7) * (gx >> 3) + (int)(blockIdx.x >> 3);
  colfwd_corr_body<L1, MODE>(x, ldx, N, b, np, logL, log2, tcol, Z, ft, r, part, rpad, cb, blockIdx.y);
}

// U laid out for colfwd_corr_body's A operand: per (column block, step, U
// tile jt) 512 values, lane (m, g) holding U[n_q][16 jt + m] for
// q = 32 t + 8 g + e, n_q = 16 cb + q / R + L2 (q % R); zero for n >= N and
// j >= r.  Mode 0: FP32, e = 4 h + i at [h][lane][i] (one 1 KB block per
// float4 load); mode 1: BF16 hi plane then lo plane, [lane][e] each.
__global__ void k_fwd_tile(const float *__restrict__ U, int64_t ldu, int N, int r, int log2, int R, int njt, int mode,
                           void *__restrict__ out, int64_t steps) {
  const int64_t total = steps * 512;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t st = i >> 9;  // (cb T + t) njt + jt
    const int w = (int)(i & 511);
    int lane, e;
    if (mode == 0) {
      lane = (w & 255) >> 2;
      e = 4 * (w >> 8) + (w & 3);
    } else {
      lane = w >> 3;
      e = w & 7;
    }
    const int jt = (int)(st % njt);
    const int64_t ct = st / njt;
    const int T = 8 * R / 16;  // Q / 32 with Q = 16 R
    const int t = (int)(ct % T);
    const int64_t cb = ct / T;
    const int m = lane & 15, g = lane >> 4;
    const int q = 32 * t + 8 * g + e;
    const int64_t n = cb * 16 + q / R + ((int64_t)(q % R) << log2);
    const int j = 16 * jt + m;
    const float u = (j < r && n < N) ? U[(int64_t)j * ldu + n] : 0.f;
    if (mode == 0) {
      static_cast<float *>(out)[i] = u;
    } else {
      const __bf16 h = (__bf16)u;
      __bf16 *o = static_cast<__bf16 *>(out) + st * 1024;
      o[w] = h;
      o[512 + w] = (__bf16)(u - (float)h);
    }
  }
}

bool colfwd_corr_ok(const FftGeom &g, int r) {
  return g.v2 && !g.single() && (g.log1 == 4 || g.log1 == 5) && r >= 1 && r <= 32;
}

int colfwd_corr_chunks(const FftGeom &g) { return 1 << (g.log2 - 4); }

static int64_t fwd_tile_steps(const FftGeom &g, int r) {
  const int R = (1 << g.log1) / 2;
  return ((int64_t)1 << (g.log2 - 4)) * (16 * R / 32) * ((r + 15) / 16);
}

size_t fwd_tile_bytes(const FftGeom &g, int r) { return (size_t)fwd_tile_steps(g, r) * 2048; }

hipError_t build_fwd_tile(const float *U, int64_t ldu, int N, int r, const FftGeom &g, int mode, void *out,
                          hipStream_t st) {
  if (!colfwd_corr_ok(g, r)) return hipErrorInvalidValue;
  const int64_t steps = fwd_tile_steps(g, r);
  const int64_t blocks = std::min<int64_t>((steps * 512 + 255) / 256, 65536);
  SLP_LAUNCH("fwd_tile", k_fwd_tile, dim3((unsigned)blocks), dim3(256), 0, st, U, ldu, N, r, g.log2,
             (1 << g.log1) / 2, (r + 15) / 16, mode, out, steps);
  return hipGetLastError();
}

hipError_t colfwd_corr(const float *x, int64_t ldx, int64_t N, int64_t b, const FftGeom &g,
                       const FftTables<float> &tb, cpx<float> *Z, const void *ft, int r, int mode, float *part,
                       hipStream_t st) {
  if (!colfwd_corr_ok(g, r) || (mode != 0 && mode != 1)) return hipErrorInvalidValue;
  const int64_t np = (b + 1) / 2;
  const int64_t pwg = 4 * kFcWaves;  // pairs per workgroup
  if (np == 0) return hipSuccess;
  if ((np + pwg - 1) / pwg > 65535) return hipErrorInvalidValue;
  const dim3 grid(1u << (g.log2 - 4), (unsigned)((np + pwg - 1) / pwg));
  const int rpad = corr_rpad(r);
#define SLP_CFC(L1, M, NAME)                                                                                        \
  SLP_LAUNCH(NAME, (k_colfwd_corr<L1, M>), grid, dim3(64 * kFcWaves), 0, st, x, ldx, (int)N, (int)b, (int)np,     \
             g.logL, g.log2, tb.col, Z, ft, r, part, rpad)
  if (g.log1 == 5) {
    if (mode) SLP_CFC(32, 1, "col_fwd_corr_bf16x3");
    else SLP_CFC(32, 0, "col_fwd_corr");
  } else {
    if (mode) SLP_CFC(16, 1, "col_fwd_corr_bf16x3");
    else SLP_CFC(16, 0, "col_fwd_corr");
  }
#undef SLP_CFC
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Grouped launches: workgroup -> (plan, local workgroup) by binary search over
// the span's start offsets, then the same bodies as the single-plan kernels.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int group_slot(const int *__restrict__ start, int m, int bid) {
  int lo = 0, hi = m;  // start[lo] <= bid < start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= bid) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int R1, int R2, int R3, bool CORR>
__global__ __launch_bounds__(R2 *R3) void k_single2_group(const GroupPlan *__restrict__ gp,
                                                          const int *__restrict__ idx,
                                                          const int *__restrict__ start, int m) {
  const int q = group_slot(start, m, blockIdx.x);
  const GroupPlan &P = gp[idx[q]];
  single_body<float, R1, R2, R3, CORR>(P.x, P.ldx, P.y, P.ldy, P.N, P.b, P.rt1, P.rt2, P.chat, P.beta, P.gl, P.corr,
                                       (int)blockIdx.x - start[q]);
}

template <int L1>
__global__ __launch_bounds__(256) void k_colinv2_group(const GroupPlan *__restrict__ gp, const int *__restrict__ idx,
                                                       const int *__restrict__ start, int m) {
  const int q = group_slot(start, m, blockIdx.x);
  const GroupPlan &P = gp[idx[q]];
  const int w = (int)blockIdx.x - start[q], sh = P.log2 - 8;  // 2^sh column blocks of 256
  colinv_body<float, L1>(P.Z, P.N, P.b, 0, P.logL, P.log2, P.tcol, P.y, P.ldy, w & ((1 << sh) - 1), w >> sh);
}

template <int L1>
__global__ __launch_bounds__(256) void k_colfwd2_group(const GroupPlan *__restrict__ gp, const int *__restrict__ idx,
                                                       const int *__restrict__ start, int m) {
  const int q = group_slot(start, m, blockIdx.x);
  const GroupPlan &P = gp[idx[q]];
  const int w = (int)blockIdx.x - start[q], sh = P.log2 - 8;  // 2^sh column blocks of 256
  colfwd_body<float, L1>(P.x, P.ldx, P.N, P.b, 0, P.logL, P.log2, P.tcol, P.Z, w & ((1 << sh) - 1), w >> sh);
}

template <int R1, int R2, int R3>
__global__ __launch_bounds__(R2 *R3) void k_row2_group(const GroupPlan *__restrict__ gp, const int *__restrict__ idx,
                                                       const int *__restrict__ start, int m) {
  const int q = group_slot(start, m, blockIdx.x);
  const GroupPlan &P = gp[idx[q]];
  const int w = (int)blockIdx.x - start[q];
  row_body<float, R1, R2, R3>(P.Z, P.logL, P.log2, P.rt1, P.rt2, P.chat, P.beta, P.gl, w & ((1 << P.log1) - 1),
                              w >> P.log1);
}

// ONE: the single-step contraction (L1 = 32, one pair per lane, rank <= 32),
// as the single-plan launch takes it for those plans, so that the grouped
// call reproduces the plan's own calls bit for bit.
template <int L1, int MODE, int CW, int PPL, bool ONE = false>
__global__ __launch_bounds__(64 * CW, L1 >= 32 ? 3 : kCicWaves) void k_colinv_corr_group(const GroupPlan *__restrict__ gp,
                                                               const int *__restrict__ idx,
                                                               const int *__restrict__ start, int m) {
  const int q = group_slot(start, m, blockIdx.x);
  const GroupPlan &P = gp[idx[q]];
  const int w = (int)blockIdx.x - start[q], sh = P.log2 - 4;  // 2^sh column blocks of 16
  colinv_corr_body<L1, MODE, CW, PPL, false, ONE>(P.Z, P.N, P.b, 0, P.np, P.logL, P.log2, P.tcol, P.y, P.ldy,
                                                  P.corr.ut, P.corr.r, P.rp, P.corr.dC, w & ((1 << sh) - 1), w >> sh);
}

template <int L1, int MODE>
__global__ __launch_bounds__(64 * kFcWaves, 3) void k_colfwd_corr_group(const GroupPlan *__restrict__ gp,
                                                                     const int *__restrict__ idx,
                                                                     const int *__restrict__ start, int m) {
  const int q = group_slot(start, m, blockIdx.x);
  const GroupPlan &P = gp[idx[q]];
  const int w = (int)blockIdx.x - start[q], sh = P.log2 - 4;  // 2^sh column blocks of 16
  colfwd_corr_body<L1, MODE>(P.x, P.ldx, P.N, P.b, P.np, P.logL, P.log2, P.tcol, P.Z, P.ftile, P.corr.r, P.part,
                             P.rpad, w & ((1 << sh) - 1), w >> sh);
}

// Row twiddle tables: rt1[k1 T + t] = W_L2^{t k1}, rt2[k2 R3 + m'] = W_T^{m' k2}.
template <typename R>
__global__ void k_row_twiddles(cpx<R> *__restrict__ rt1, cpx<R> *__restrict__ rt2, int R1, int R2, int R3) {
  const int T = R2 * R3, L2 = R1 * T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L2) {
    const int k1 = i / T, t = i % T;
    const int m = (t * k1) % L2;
    double sn, cs;
    sincospi(2.0 * (double)m / (double)L2, &sn, &cs);
    rt1[i] = cpx<R>{(R)cs, (R)(-sn)};
  }
  if (i < T) {
    const int k2 = i / R3, mp = i % R3;
    const int m = (mp * k2) % T;
    double sn, cs;
    sincospi(2.0 * (double)m / (double)T, &sn, &cs);
    rt2[i] = cpx<R>{(R)cs, (R)(-sn)};
  }
}

// Column-pass twiddles: tc[k1 L2 + n2] = W_L^{k1 n2} (k1 < L1, n2 < L2), so a
// lane's factor for row k1 is one coalesced load.
template <typename R>
__global__ void k_col_twiddles(cpx<R> *__restrict__ tc, int log2, int logL) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ((int64_t)1 << logL)) return;
  const int64_t k1 = i >> log2, n2 = i & (((int64_t)1 << log2) - 1);
  double sn, cs;
  sincospi(ldexp((double)(k1 * n2), 1 - logL), &sn, &cs);
  tc[i] = cpx<R>{(R)cs, (R)(-sn)};
}

template <typename R>
hipError_t build_col_table(const FftGeom &g, cpx<R> *tc, hipStream_t st) {
  if (!g.v2 || g.single()) return hipSuccess;
  const int64_t L = (int64_t)1 << g.logL;
  hipLaunchKernelGGL(k_col_twiddles<R>, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, st, tc, g.log2, g.logL);
  return hipGetLastError();
}

template <typename R>
hipError_t build_row_tables(const FftGeom &g, cpx<R> *rt1, cpx<R> *rt2, hipStream_t st) {
  if (!g.v2) return hipSuccess;
  const int L2 = g.R1 * g.R2 * g.R3;
  hipLaunchKernelGGL(k_row_twiddles<R>, dim3((L2 + 255) / 256), dim3(256), 0, st, rt1, rt2, g.R1, g.R2, g.R3);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------

template <typename R, int R1, int R2, int R3>
static void launch_row(dim3 grid, hipStream_t st, cpx<R> *Z, const FftGeom &g, const FftTables<R> &tb, R beta,
                       R gl, const RowSum *rs = nullptr) {
  if constexpr (sizeof(R) == 4) {
    if (rs && rs->blocks > 0) {
      RowSum a = *rs;
      a.ey = (int)((a.blocks + grid.x - 1) / grid.x);
      SLP_LAUNCH("row_conv", (k_row2_sum<R1, R2, R3>), dim3(grid.x, grid.y + (unsigned)a.ey), dim3(R2 * R3), 0, st,
                 Z, g.logL, g.log2, tb.row1, tb.row2, tb.chat, beta, gl, a);
      return;
    }
  }
  SLP_LAUNCH(sizeof(R) == 4 ? "row_conv" : "row_conv_f64", (k_row2<R, R1, R2, R3>), grid, dim3(R2 * R3), 0, st, Z,
             g.logL, g.log2, tb.row1, tb.row2, tb.chat, beta, gl);
}

template <typename R, int R1, int R2, int R3>
static void launch_single(int64_t np, hipStream_t st, const R *x, int64_t ldx, R *y, int64_t ldy, int N, int b,
                          const FftTables<R> &tb, R beta, R gl, const Corr<R> &c) {
  if (c.r > 0) {
    SLP_LAUNCH("conv_single_corr", (k_single2<R, R1, R2, R3, true>), dim3((unsigned)np), dim3(R2 * R3), 0, st, x,
               ldx, y, ldy, N, b, tb.row1, tb.row2, tb.chat, beta, gl, c);
  } else {
    SLP_LAUNCH(sizeof(R) == 4 ? "conv_single" : "conv_single_f64", (k_single2<R, R1, R2, R3, false>),
               dim3((unsigned)np), dim3(R2 * R3), 0, st, x, ldx, y, ldy, N, b, tb.row1, tb.row2, tb.chat, beta, gl,
               c);
  }
}

template <typename R, int L1, bool EVEN = false>
static void launch_cols(bool fwd, dim3 grid, hipStream_t st, const R *x, int64_t ldx, R *y, int64_t ldy, int N,
                        int b, int p0, const FftGeom &g, const FftTables<R> &tb, cpx<R> *Z) {
  if (fwd && EVEN) {
    SLP_LAUNCH("col_fwd_even", (k_colfwd2_even<R, L1>), grid, dim3(256), 0, st, x, ldx, N, b, p0, g.logL, g.log2,
               tb.col, Z);
  } else if (fwd) {
    SLP_LAUNCH(sizeof(R) == 4 ? "col_fwd" : "col_fwd_f64", (k_colfwd2<R, L1>), grid, dim3(256), 0, st, x, ldx, N, b,
               p0, g.logL, g.log2, tb.col, Z);
  } else if (EVEN) {
    SLP_LAUNCH("col_inv_even", (k_colinv2_even<R, L1>), grid, dim3(256), 0, st, Z, N, b, p0, g.logL, g.log2, tb.col,
               y, ldy);
  } else {
    SLP_LAUNCH(sizeof(R) == 4 ? "col_inv" : "col_inv_f64", (k_colinv2<R, L1>), grid, dim3(256), 0, st, Z, N, b, p0,
               g.logL, g.log2, tb.col, y, ldy);
  }
}

// Long columns: (A, B) and columns per workgroup CB with L1 CB elements of
// LDS within 64 KB.
template <typename R, int A, int B, int CB, bool EVEN = false>
static void launch_cols_lds(bool fwd, hipStream_t st, const R *x, int64_t ldx, R *y, int64_t ldy, int N, int b,
                            int p0, int np, const FftGeom &g, const FftTables<R> &tb, cpx<R> *Z) {
  const dim3 grid((1u << g.log2) / CB, (unsigned)np), block(CB * A);
  if (fwd) {
    SLP_LAUNCH(EVEN ? "col_fwd_even" : sizeof(R) == 4 ? "col_fwd" : "col_fwd_f64", (k_colfwd_lds<R, A, B, CB, EVEN>),
               grid, block, 0, st, x, ldx, N, b, p0, g.logL, g.log2, tb.col, Z);
  } else {
    SLP_LAUNCH(EVEN ? "col_inv_even" : sizeof(R) == 4 ? "col_inv" : "col_inv_f64", (k_colinv_lds<R, A, B, CB, EVEN>),
               grid, block, 0, st, Z, N, b, p0, g.logL, g.log2, tb.col, y, ldy);
  }
}

template <typename R, bool EVEN = false>
static bool dispatch_cols(bool fwd, dim3 grid, hipStream_t st, const R *x, int64_t ldx, R *y, int64_t ldy, int N,
                          int b, int p0, const FftGeom &g, const FftTables<R> &tb, cpx<R> *Z) {
  const int np = (int)grid.y;
  if (g.log1 >= 6) {
    constexpr bool f32 = sizeof(R) == 4;
    switch (g.log1) {
      case 6: launch_cols_lds<R, 8, 8, 32, EVEN>(fwd, st, x, ldx, y, ldy, N, b, p0, np, g, tb, Z); return true;
      case 7: launch_cols_lds<R, 8, 16, 32, EVEN>(fwd, st, x, ldx, y, ldy, N, b, p0, np, g, tb, Z); return true;
      case 8: launch_cols_lds<R, 16, 16, 16, EVEN>(fwd, st, x, ldx, y, ldy, N, b, p0, np, g, tb, Z); return true;
      case 9:
        if (f32) launch_cols_lds<R, 16, 32, 16, EVEN>(fwd, st, x, ldx, y, ldy, N, b, p0, np, g, tb, Z);
        else launch_cols_lds<R, 16, 32, 8, EVEN>(fwd, st, x, ldx, y, ldy, N, b, p0, np, g, tb, Z);
        return true;
      default: return false;
    }
  }
  switch (g.log1) {
    case 1: launch_cols<R, 2, EVEN>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    case 2: launch_cols<R, 4, EVEN>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    case 3: launch_cols<R, 8, EVEN>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    case 4: launch_cols<R, 16, EVEN>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    case 5: launch_cols<R, 32, EVEN>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    default: return false;
  }
}

// Fused pass C launch shape: PPL pairs per lane, CW wavefronts per workgroup
// (4 PPL CW pairs of one column block, whose U tile they share through the
// caches).  SLEPIAN_CIC_SHAPE = "PPLxCW" (1x8, 1x4, 2x4) overrides the
// default for tuning.
struct CicShape {
  int ppl = 1, cw = 4;
  bool set = false;  // from the override
};

// the grouped launches use one pair per lane and 4 or 8 wavefronts (tuned)
constexpr int kGroupCicPPL = 1;

static CicShape cic_shape() {
  static const CicShape sh = [] {
    CicShape c;
    if (const char *e = std::getenv("SLEPIAN_CIC_SHAPE")) {
      int p = 0, w = 0;
      if (std::sscanf(e, "%dx%d", &p, &w) == 2 && ((p == 1 && (w == 4 || w == 8)) || (p == 2 && w == 4))) {
        c.ppl = p;
        c.cw = w;
        c.set = true;
      }
    }
    return c;
  }();
  return sh;
}

int colinv_corr_rp(int r, int mode) { return mode == 0 ? (r + 15) / 16 * 16 : (r + 31) / 32 * 32; }

// L1 = 32 keeps 64 complex inputs per lane on top of the accumulators; there
// the plain pass plus the separate matrix-core update is faster.
bool colinv_corr_ok(const FftGeom &g, int64_t ldy, int64_t b, int r) {
  // tuning override: SLEPIAN_CIC_MAXLOG1 (4 or 5), the largest L1 = 2^log1
  // fused, unless the plan was tuned (g.cicmax)
  static const int maxlog1 = [] {
    const char *e = std::getenv("SLEPIAN_CIC_MAXLOG1");
    return e && std::atoi(e) == 5 ? 5 : 4;
  }();
  const int mx = g.cicmax ? g.cicmax : maxlog1;
  // the pass addresses y and dC by 32-bit byte offsets from a wavefront's base
  const bool fits = ldy < ((int64_t)1 << 25) && (int64_t)colinv_corr_rp(r, 1) * b < ((int64_t)1 << 29);
  return g.log1 >= 1 && g.log1 <= mx && fits;
}

bool colinv_corr_tiled(const FftGeom &g) { return colinv_corr_ok(g, 1, 1, 1); }

bool colinv_corr_one(int log1, int rp) { return log1 == 5 && rp == 32; }

template <int L1, int MODE, int CW, int PPL, bool EVEN = false>
static void launch_cic(hipStream_t st, const cpx<float> *Z, int N, int b, int p0, int np, const FftGeom &g,
                       const FftTables<float> &tb, float *y, int64_t ldy, const Corr<float> &c, int rp) {
  constexpr int PW = 4 * PPL * CW;  // pairs per workgroup
  const dim3 grid((1u << g.log2) / 16, (unsigned)((np + PW - 1) / PW));
  // L1 = 32, one pair per lane, rank <= 32: the single-step contraction
  // (same bits; with two pairs per lane its registers would spill)
  if constexpr (L1 >= 32 && !EVEN && PPL == 1) {
    if (colinv_corr_one(g.log1, rp)) {
      SLP_LAUNCH(MODE ? "col_inv_corr_bf16x3" : "col_inv_corr", (k_colinv_corr<L1, MODE, CW, PPL, false, true>), grid,
                 dim3(64 * CW), 0, st, Z, N, b, p0, np, g.logL, g.log2, tb.col, y, ldy, c.ut, c.r, rp, c.dC);
      return;
    }
  }
  SLP_LAUNCH(MODE ? (EVEN ? "col_inv_even_corr_bf16x3" : "col_inv_corr_bf16x3") : (EVEN ? "col_inv_even_corr" : "col_inv_corr"),
             (k_colinv_corr<L1, MODE, CW, PPL, EVEN>), grid, dim3(64 * CW),
             0, st, Z, N, b, p0, np, g.logL, g.log2, tb.col, y, ldy, c.ut, c.r, rp, c.dC);
}

template <int L1, int MODE, bool EVEN = false>
static void launch_cic_shape(hipStream_t st, const cpx<float> *Z, int N, int b, int p0, int np, const FftGeom &g,
                             const FftTables<float> &tb, float *y, int64_t ldy, const Corr<float> &c, int rp) {
  // the even-row pass (fast factorization, update of rank r1 + r, about three
  // times the projection's) re-reads a larger U tile per pair group; two pairs
  // per lane halve the groups (measured 77 -> 53 us at rank 91)
  CicShape sh = cic_shape();
  if (g.cic >= 1 && g.cic <= 3) {
    sh.ppl = g.cic == 3 ? 2 : 1;
    sh.cw = g.cic == 2 ? 8 : 4;
    sh.set = true;
  }
  if (EVEN && !sh.set) {
    sh.ppl = 2;
    sh.cw = 4;
  }
  if (sh.ppl == 1 && sh.cw == 8) launch_cic<L1, MODE, 8, 1, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c, rp);
  else if (sh.ppl == 1) launch_cic<L1, MODE, 4, 1, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c, rp);
  else launch_cic<L1, MODE, 4, 2, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c, rp);
}

template <int MODE, bool EVEN = false>
static bool launch_cic_mode(hipStream_t st, const cpx<float> *Z, int N, int b, int p0, int np, const FftGeom &g,
                            const FftTables<float> &tb, float *y, int64_t ldy, const Corr<float> &c) {
  const int rp = colinv_corr_rp(c.r, MODE);
  if (!c.ut) return false;
  switch (g.log1) {
    case 1: launch_cic_shape<2, MODE, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    case 2: launch_cic_shape<4, MODE, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    case 3: launch_cic_shape<8, MODE, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    case 4: launch_cic_shape<16, MODE, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    case 5: launch_cic_shape<32, MODE, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    default: return false;  // larger L1: the caller does the update separately
  }
}

template <bool EVEN = false>
static bool launch_colinv_corr(hipStream_t st, const cpx<float> *Z, int N, int b, int p0, int np, const FftGeom &g,
                               const FftTables<float> &tb, float *y, int64_t ldy, const Corr<float> &c) {
  return c.mode == 0 ? launch_cic_mode<0, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c)
                     : launch_cic_mode<1, EVEN>(st, Z, N, b, p0, np, g, tb, y, ldy, c);
}

#define SLP_ROW_SHAPES(X) \
  X(8, 8, 8)              \
  X(16, 8, 8)             \
  X(16, 16, 8)            \
  X(16, 16, 16)           \
  X(32, 16, 16)

// fwd_done: pass A has already written Z (one slice; x is not read).  rs: the
// chunk sum the row pass carries (or null).
template <typename R>
static hipError_t conv_apply_impl(const R *x, int64_t ldx, R *y, int64_t ldy, int64_t N, int64_t b,
                                  const FftGeom &g, const FftTables<R> &tb, R beta, R gamma, const Corr<R> &corr,
                                  cpx<R> *Z, int64_t slice_pairs, bool fwd_done, hipStream_t st,
                                  const RowSum *rs = nullptr) {
  const int64_t pairs = (b + 1) / 2;
  if (pairs == 0) return hipSuccess;
  const R gl = gamma / (R)((int64_t)1 << g.logL);
  if (g.single()) {
    for (int64_t p0 = 0; p0 < pairs; p0 += 65535) {
      const int64_t np = pairs - p0 < 65535 ? pairs - p0 : 65535;
      const R *xs = x + 2 * p0 * ldx;
      R *ys = y + 2 * p0 * ldy;
      const int bs = (int)(b - 2 * p0 < 2 * np ? b - 2 * p0 : 2 * np);
      bool ok = false;
#define SLP_SINGLE(A, B, C)                                                                                  \
  if (!ok && g.R1 == A && g.R2 == B && g.R3 == C) {                                                           \
    if constexpr (sizeof(R) == 4 || A * B * C <= 4096) {                                                      \
      launch_single<R, A, B, C>(np, st, xs, ldx, ys, ldy, (int)N, bs, tb, beta, gl, corr);                    \
      ok = true;                                                                                              \
    }                                                                                                         \
  }
      SLP_ROW_SHAPES(SLP_SINGLE)
#undef SLP_SINGLE
      if (!ok) return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  for (int64_t p0 = 0; p0 < pairs; p0 += slice_pairs) {
    const int64_t np = pairs - p0 < slice_pairs ? pairs - p0 : slice_pairs;
    const dim3 gcol((1u << g.log2) / 256, (unsigned)np);
    const dim3 grow(1u << g.log1, (unsigned)np);
    if (!fwd_done && !dispatch_cols<R>(true, gcol, st, x, ldx, y, ldy, (int)N, (int)b, (int)p0, g, tb, Z))
      return hipErrorInvalidValue;
    bool ok = false;
#define SLP_ROW(A, B, C)                                                                                     \
  if (!ok && g.R1 == A && g.R2 == B && g.R3 == C) {                                                           \
    if constexpr (sizeof(R) == 4 || A * B * C <= 4096) {                                                      \
      launch_row<R, A, B, C>(grow, st, Z, g, tb, beta, gl, rs);                                               \
      ok = true;                                                                                              \
    }                                                                                                         \
  }
    SLP_ROW_SHAPES(SLP_ROW)
#undef SLP_ROW
    if (!ok) return hipErrorInvalidValue;
    if constexpr (sizeof(R) == 4) {
      if (corr.dC) {
        if (!launch_colinv_corr(st, Z, (int)N, (int)b, (int)p0, (int)np, g, tb, y, ldy, corr))
          return hipErrorInvalidValue;
        continue;
      }
    }
    if (!dispatch_cols<R>(false, gcol, st, x, ldx, y, ldy, (int)N, (int)b, (int)p0, g, tb, Z))
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename R>
hipError_t conv_apply_v2(const R *x, int64_t ldx, R *y, int64_t ldy, int64_t N, int64_t b, const FftGeom &g,
                         const FftTables<R> &tb, R beta, R gamma, const Corr<R> &corr, cpx<R> *Z, int64_t slice_pairs,
                         hipStream_t st) {
  return conv_apply_impl<R>(x, ldx, y, ldy, N, b, g, tb, beta, gamma, corr, Z, slice_pairs, false, st);
}

hipError_t conv_rows_inv(float *y, int64_t ldy, int64_t N, int64_t b, const FftGeom &g, const FftTables<float> &tb,
                         float beta, float gamma, const Corr<float> &corr, cpx<float> *Z, const RowSum *rs,
                         hipStream_t st) {
  if (g.single() || !g.v2) return hipErrorInvalidValue;
  const int64_t pairs = (b + 1) / 2;
  return conv_apply_impl<float>(nullptr, 0, y, ldy, N, b, g, tb, beta, gamma, corr, Z, pairs > 0 ? pairs : 1, true,
                                st, rs);
}

// ---- length-N DFT bins for the fast factorization (Section 1.3) ----
//
// With L = 2N, bin K = 2k of the length-L transform of the zero-padded pair
// z = x1 + i x2 is bin k of its length-N transform.  The bins kept are
// |k| <= M = (kf - 1)/2, stored per pair at slot M + k (k < 0 wraps to
// K = L + 2k).  Within a row the stage-3 value m of job q sits at row
// frequency kr = d1 + R1 d2 + R1 R2 m (q -> g = t + T q, d1 = g / R2,
// d2 = g % R2), full frequency K = k1c + L1 kr.

// slot of full frequency K (even), or -1 if the bin is not kept
__device__ __forceinline__ int bin_slot(int64_t K, int64_t N, int M) {
  const int64_t k = K >> 1;
  if (k <= M) return (int)(M + k);
  if (k >= N - M) return (int)(M - (N - k));
  return -1;
}

template <int R1, int R2, int R3>
__device__ __forceinline__ int64_t row_freq(int q, int m) {
  constexpr int T = R2 * R3;
  const int g = threadIdx.x + T * q;
  return (int64_t)(g / R2) + (int64_t)R1 * (g % R2) + (int64_t)R1 * R2 * m;
}

// Workgroup -> (even row h, pair pl) for the bins row passes.  Workgroups
// are dealt to the 8 XCDs round robin by linear id; w = 8 (h + R g) + q with
// pair pl = 8 g + q puts all R = L1/2 even rows of a pair on one XCD, so the
// rows' interleaved bins (slots M + h + R kr) meet in one L2.  Workgroups
// past the last pair exit at once (before any barrier).
__device__ __forceinline__ bool bins_row_pair(int R, int np, int &h, int &pl) {
  const int w = blockIdx.x, q = w & 7, rest = w >> 3;
  h = rest % R;
  pl = (rest / R) * 8 + q;
  return pl < np;
}

// Forward row transforms of the even rows k1c = 2h of pair pl, kept bins
// written to Zb[pl][slot].
template <int R1, int R2, int R3>
__global__ __launch_bounds__(R2 *R3) void k_row_bins(const cpx<float> *__restrict__ Z, int logL, int log1, int log2,
                                                    const cpx<float> *__restrict__ rt1,
                                                    const cpx<float> *__restrict__ rt2, cpx<float> *__restrict__ Zb,
                                                    int kf, int np) {
  using RS = RowShape<R1, R2, R3>;
  __shared__ cpx<float> S[RS::LDS];
  __shared__ cpx<float> rt2s[R2 * (R3 + 1)];
  int h, pl;
  if (!bins_row_pair(1 << (log1 - 1), np, h, pl)) return;
  const int k1c = 2 * h;
  const cpx<float> *row = Z + ((int64_t)pl << logL) + ((int64_t)k1c << log2);
  const int t = threadIdx.x;
  cpx<float> v[R1];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) v[n1] = row[t + RS::T * n1];
  cpx<float> tw1[R1];
  load_tw1<float, R1, R2, R3>(tw1, rt1);
  stage_rt2<float, R1, R2, R3>(rt2s, rt2);
  const int64_t N = (int64_t)1 << (logL - 1);
  const int M = (kf - 1) / 2;
  cpx<float> *out = Zb + (int64_t)pl * kf;
  row_conv_core<float, R1, R2, R3, 1>(v, S, tw1, rt2s, [&](cpx<float> *z, int q) {
#pragma unroll
    for (int m = 0; m < R3; ++m) {
      const int sl = bin_slot(k1c + (row_freq<R1, R2, R3>(q, m) << log1), N, M);
      if (sl >= 0) out[sl] = z[m];
    }
  });
}

// Inverse row transforms of the even rows k1c = 2h of pair pl from the kept
// bins (zero elsewhere; workgroups mapped as in k_row_bins).  Odd rows hold
// no even frequency; they are neither written here nor read by the inverse
// column pass that follows.
template <int R1, int R2, int R3>
__global__ __launch_bounds__(R2 *R3) void k_row_from_bins(const cpx<float> *__restrict__ Zb, int kf, int logL,
                                                         int log1, int log2, const cpx<float> *__restrict__ rt1,
                                                         const cpx<float> *__restrict__ rt2,
                                                         cpx<float> *__restrict__ Z, int np) {
  using RS = RowShape<R1, R2, R3>;
  __shared__ cpx<float> S[RS::LDS];
  __shared__ cpx<float> rt2s[R2 * (R3 + 1)];
  int h, pl;
  if (!bins_row_pair(1 << (log1 - 1), np, h, pl)) return;
  const int k1c = 2 * h;
  cpx<float> *row = Z + ((int64_t)pl << logL) + ((int64_t)k1c << log2);
  const int t = threadIdx.x;
  cpx<float> v[R1];
  cpx<float> tw1[R1];
  load_tw1<float, R1, R2, R3>(tw1, rt1);
  stage_rt2<float, R1, R2, R3>(rt2s, rt2);
  const int64_t N = (int64_t)1 << (logL - 1);
  const int M = (kf - 1) / 2;
  const cpx<float> *in = Zb + (int64_t)pl * kf;
  row_conv_core<float, R1, R2, R3, 2>(v, S, tw1, rt2s, [&](cpx<float> *z, int q) {
#pragma unroll
    for (int m = 0; m < R3; ++m) {
      const int sl = bin_slot(k1c + (row_freq<R1, R2, R3>(q, m) << log1), N, M);
      z[m] = sl >= 0 ? in[sl] : cpx<float>{0.f, 0.f};
    }
  });
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) row[t + RS::T * n1] = v[n1];
}

// Single pass (L = R1 R2 R3): forward transform of pair blockIdx.x of x,
// kept bins to Zb.
template <int R1, int R2, int R3>
__global__ __launch_bounds__(R2 *R3) void k_single_bins(const float *__restrict__ x, int64_t ldx, int N, int b,
                                                       const cpx<float> *__restrict__ rt1,
                                                       const cpx<float> *__restrict__ rt2, cpx<float> *__restrict__ Zb,
                                                       int kf) {
  using RS = RowShape<R1, R2, R3>;
  constexpr int T = RS::T;
  __shared__ cpx<float> S[RS::LDS];
  __shared__ cpx<float> rt2s[R2 * (R3 + 1)];
  const int t = threadIdx.x, p = blockIdx.x;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const float *x0 = x + (int64_t)s0 * ldx;
  const float *x1 = x + (int64_t)(has1 ? s1 : s0) * ldx;
  cpx<float> v[R1];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    const int n = t + T * n1;
    float a = 0.f, c = 0.f;
    if (n < N) {
      a = x0[n];
      if (has1) c = x1[n];
    }
    v[n1] = cpx<float>{a, c};
  }
  cpx<float> tw1[R1];
  load_tw1<float, R1, R2, R3>(tw1, rt1);
  stage_rt2<float, R1, R2, R3>(rt2s, rt2);
  const int M = (kf - 1) / 2;
  cpx<float> *out = Zb + (int64_t)p * kf;
  row_conv_core<float, R1, R2, R3, 1>(v, S, tw1, rt2s, [&](cpx<float> *z, int q) {
#pragma unroll
    for (int m = 0; m < R3; ++m) {
      const int64_t K = row_freq<R1, R2, R3>(q, m);
      const int sl = (K & 1) ? -1 : bin_slot(K, N, M);
      if (sl >= 0) out[sl] = z[m];
    }
  });
}

// Single pass: inverse transform of pair blockIdx.x from its kept bins,
// samples n < N to y.
template <int R1, int R2, int R3>
__global__ __launch_bounds__(R2 *R3) void k_single_from_bins(const cpx<float> *__restrict__ Zb, int kf,
                                                            float *__restrict__ y, int64_t ldy, int N, int b,
                                                            const cpx<float> *__restrict__ rt1,
                                                            const cpx<float> *__restrict__ rt2) {
  using RS = RowShape<R1, R2, R3>;
  constexpr int T = RS::T;
  __shared__ cpx<float> S[RS::LDS];
  __shared__ cpx<float> rt2s[R2 * (R3 + 1)];
  const int t = threadIdx.x, p = blockIdx.x;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  cpx<float> tw1[R1];
  load_tw1<float, R1, R2, R3>(tw1, rt1);
  stage_rt2<float, R1, R2, R3>(rt2s, rt2);
  const int M = (kf - 1) / 2;
  const cpx<float> *in = Zb + (int64_t)p * kf;
  cpx<float> v[R1];
  row_conv_core<float, R1, R2, R3, 2>(v, S, tw1, rt2s, [&](cpx<float> *z, int q) {
#pragma unroll
    for (int m = 0; m < R3; ++m) {
      const int64_t K = row_freq<R1, R2, R3>(q, m);
      const int sl = (K & 1) ? -1 : bin_slot(K, N, M);
      z[m] = sl >= 0 ? in[sl] : cpx<float>{0.f, 0.f};
    }
  });
  float *y0 = y + (int64_t)s0 * ldy;
  float *y1 = y + (int64_t)s1 * ldy;
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    const int n = t + T * n1;
    if (n < N) {
      y0[n] = v[n1].x;
      if (has1) y1[n] = v[n1].y;
    }
  }
}

bool dft_bins_ok(const FftGeom &g, int64_t N) {
  if (!g.v2 || ((int64_t)1 << g.logL) != 2 * N) return false;
  bool ok = false;
#define SLP_BOK(A, B, C) ok = ok || (g.R1 == A && g.R2 == B && g.R3 == C);
  SLP_ROW_SHAPES(SLP_BOK)
#undef SLP_BOK
  return ok && (g.single() || g.log1 <= 9);
}

hipError_t dft_bins_fwd(const float *x, int64_t ldx, int64_t N, int64_t b, const FftGeom &g,
                        const FftTables<float> &tb, cpx<float> *Z, int64_t slice_pairs, cpx<float> *Zb, int kf,
                        hipStream_t st) {
  const int64_t pairs = (b + 1) / 2;
  if (pairs == 0) return hipSuccess;
  if (!dft_bins_ok(g, N)) return hipErrorInvalidValue;
  if (g.single()) {
    for (int64_t p0 = 0; p0 < pairs; p0 += 65535) {
      const int64_t np = std::min<int64_t>(65535, pairs - p0);
      const int bs = (int)std::min<int64_t>(b - 2 * p0, 2 * np);
#define SLP_SB(A, B, C)                                                                                        \
  if (g.R1 == A && g.R2 == B && g.R3 == C)                                                                      \
    SLP_LAUNCH("dft_bins_single", (k_single_bins<A, B, C>), dim3((unsigned)np), dim3(B * C), 0, st,           \
               x + 2 * p0 * ldx, ldx, (int)N, bs, tb.row1, tb.row2, Zb + p0 * kf, kf);
      SLP_ROW_SHAPES(SLP_SB)
#undef SLP_SB
    }
    return hipGetLastError();
  }
  for (int64_t p0 = 0; p0 < pairs; p0 += slice_pairs) {
    const int64_t np = std::min<int64_t>(slice_pairs, pairs - p0);
    const dim3 gcol((1u << g.log2) / 256, (unsigned)np);
    if (!dispatch_cols<float, true>(true, gcol, st, x, ldx, nullptr, 0, (int)N, (int)b, (int)p0, g, tb, Z))
      return hipErrorInvalidValue;
    const dim3 grow((unsigned)(((np + 7) / 8) * 8 << (g.log1 - 1)));
#define SLP_RB(A, B, C)                                                                                         \
  if (g.R1 == A && g.R2 == B && g.R3 == C)                                                                       \
    SLP_LAUNCH("dft_bins_row", (k_row_bins<A, B, C>), grow, dim3(B * C), 0, st, Z, g.logL, g.log1, g.log2,     \
               tb.row1, tb.row2, Zb + p0 * kf, kf, (int)np);
    SLP_ROW_SHAPES(SLP_RB)
#undef SLP_RB
  }
  return hipGetLastError();
}

hipError_t dft_bins_inv(const cpx<float> *Zb, int kf, float *y, int64_t ldy, int64_t N, int64_t b,
                        const FftGeom &g, const FftTables<float> &tb, cpx<float> *Z, int64_t slice_pairs,
                        const Corr<float> &corr, hipStream_t st) {
  const int64_t pairs = (b + 1) / 2;
  if (pairs == 0) return hipSuccess;
  if (!dft_bins_ok(g, N)) return hipErrorInvalidValue;
  if (g.single()) {
    for (int64_t p0 = 0; p0 < pairs; p0 += 65535) {
      const int64_t np = std::min<int64_t>(65535, pairs - p0);
      const int bs = (int)std::min<int64_t>(b - 2 * p0, 2 * np);
#define SLP_SI(A, B, C)                                                                                        \
  if (g.R1 == A && g.R2 == B && g.R3 == C)                                                                      \
    SLP_LAUNCH("dft_from_bins_single", (k_single_from_bins<A, B, C>), dim3((unsigned)np), dim3(B * C), 0, st, \
               Zb + p0 * kf, kf, y + 2 * p0 * ldy, ldy, (int)N, bs, tb.row1, tb.row2);
      SLP_ROW_SHAPES(SLP_SI)
#undef SLP_SI
    }
    return hipGetLastError();
  }
  for (int64_t p0 = 0; p0 < pairs; p0 += slice_pairs) {
    const int64_t np = std::min<int64_t>(slice_pairs, pairs - p0);
    const dim3 grow((unsigned)(((np + 7) / 8) * 8 << (g.log1 - 1)));
#define SLP_RI(A, B, C)                                                                                         \
  if (g.R1 == A && g.R2 == B && g.R3 == C)                                                                       \
    SLP_LAUNCH("dft_from_bins_row", (k_row_from_bins<A, B, C>), grow, dim3(B * C), 0, st, Zb + p0 * kf, kf,    \
               g.logL, g.log1, g.log2, tb.row1, tb.row2, Z, (int)np);
    SLP_ROW_SHAPES(SLP_RI)
#undef SLP_RI
    if (corr.dC) {
      if (!launch_colinv_corr<true>(st, Z, (int)N, (int)b, (int)p0, (int)np, g, tb, y, ldy, corr))
        return hipErrorInvalidValue;
      continue;
    }
    const dim3 gcol((1u << g.log2) / 256, (unsigned)np);
    if (!dispatch_cols<float, true>(false, gcol, st, nullptr, 0, y, ldy, (int)N, (int)b, (int)p0, g, tb, Z))
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- grouped launch helpers ----

int64_t group_blocks_single(const GroupPlan &P) { return P.np; }
int64_t group_blocks_colfwd(const GroupPlan &P) { return (int64_t)P.np << (P.log2 - 8); }
int64_t group_blocks_row(const GroupPlan &P) { return (int64_t)P.np << P.log1; }
int64_t group_blocks_colinv(const GroupPlan &P, int cw) {
  const int pw = 4 * kGroupCicPPL * cw;
  return ((int64_t)(P.np + pw - 1) / pw) << (P.log2 - 4);
}

hipError_t group_single(int log2, bool corr, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st) {
  if (sp.m == 0) return hipSuccess;
  const dim3 grid((unsigned)sp.blocks);
  bool ok = false;
#define SLP_GSINGLE(A, B, C)                                                                                  \
  if (!ok && A * B * C == (1 << log2)) {                                                                      \
    if (corr)                                                                                                 \
      SLP_LAUNCH("single_corr_group", (k_single2_group<A, B, C, true>), grid, dim3(B * C), 0, st, gp, sp.idx, \
                 sp.start, sp.m);                                                                             \
    else                                                                                                      \
      SLP_LAUNCH("single_group", (k_single2_group<A, B, C, false>), grid, dim3(B * C), 0, st, gp, sp.idx,     \
                 sp.start, sp.m);                                                                             \
    ok = true;                                                                                                \
  }
  SLP_ROW_SHAPES(SLP_GSINGLE)
#undef SLP_GSINGLE
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t group_colfwd(int log1, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st) {
  if (sp.m == 0) return hipSuccess;
  const dim3 grid((unsigned)sp.blocks);
  switch (log1) {
#define SLP_GCF(LG, L1)                                                                                        \
  case LG:                                                                                                    \
    SLP_LAUNCH("col_fwd_group_L1_" #L1, k_colfwd2_group<L1>, grid, dim3(256), 0, st, gp, sp.idx, sp.start,  \
               sp.m);                                                                                         \
    break;
    SLP_GCF(1, 2) SLP_GCF(2, 4) SLP_GCF(3, 8) SLP_GCF(4, 16) SLP_GCF(5, 32)
#undef SLP_GCF
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t group_colinv(int log1, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st) {
  if (sp.m == 0) return hipSuccess;
  const dim3 grid((unsigned)sp.blocks);
  switch (log1) {
#define SLP_GCV(LG, L1)                                                                                        \
  case LG:                                                                                                    \
    SLP_LAUNCH("col_inv_group_L1_" #L1, k_colinv2_group<L1>, grid, dim3(256), 0, st, gp, sp.idx, sp.start,  \
               sp.m);                                                                                         \
    break;
    SLP_GCV(1, 2) SLP_GCV(2, 4) SLP_GCV(3, 8) SLP_GCV(4, 16) SLP_GCV(5, 32)
#undef SLP_GCV
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t group_row(int log2, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st) {
  if (sp.m == 0) return hipSuccess;
  if (log2 == 13) {
    SLP_LAUNCH("row_conv_group", (k_row2_group<32, 16, 16>), dim3((unsigned)sp.blocks), dim3(256), 0, st, gp,
               sp.idx, sp.start, sp.m);
  } else if (log2 == 12) {
    SLP_LAUNCH("row_conv_group_4096", (k_row2_group<16, 16, 16>), dim3((unsigned)sp.blocks), dim3(256), 0, st, gp,
               sp.idx, sp.start, sp.m);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int64_t group_blocks_colfwd_corr(const GroupPlan &P) {
  constexpr int pwg = 4 * kFcWaves;
  return ((int64_t)(P.np + pwg - 1) / pwg) << (P.log2 - 4);
}

hipError_t group_colfwd_corr(int log1, int mode, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st) {
  if (sp.m == 0) return hipSuccess;
  const dim3 grid((unsigned)sp.blocks), block(64 * kFcWaves);
  switch (log1 * 2 + (mode ? 1 : 0)) {
    case 8:
      SLP_LAUNCH("col_fwd_corr_group_L1_16", (k_colfwd_corr_group<16, 0>), grid, block, 0, st, gp, sp.idx, sp.start,
                 sp.m);
      break;
    case 9:
      SLP_LAUNCH("col_fwd_corr_bf16x3_group_L1_16", (k_colfwd_corr_group<16, 1>), grid, block, 0, st, gp, sp.idx,
                 sp.start, sp.m);
      break;
    case 10:
      SLP_LAUNCH("col_fwd_corr_group_L1_32", (k_colfwd_corr_group<32, 0>), grid, block, 0, st, gp, sp.idx, sp.start,
                 sp.m);
      break;
    case 11:
      SLP_LAUNCH("col_fwd_corr_bf16x3_group_L1_32", (k_colfwd_corr_group<32, 1>), grid, block, 0, st, gp, sp.idx,
                 sp.start, sp.m);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int CW>
static hipError_t group_colinv_cw(int log1, int mode, bool one, const GroupPlan *gp, const GroupSpan &sp,
                                  hipStream_t st) {
  const dim3 grid((unsigned)sp.blocks), block(64 * CW);
  constexpr int PPL = kGroupCicPPL;
  static_assert(PPL == 1, "the single-step contraction takes one pair per lane");
  if (one) {
    if (log1 != 5) return hipErrorInvalidValue;
    if (mode)
      SLP_LAUNCH("col_inv_corr_bf16x3_group_L1_32", (k_colinv_corr_group<32, 1, CW, PPL, true>), grid, block, 0, st,
                 gp, sp.idx, sp.start, sp.m);
    else
      SLP_LAUNCH("col_inv_corr_group_L1_32", (k_colinv_corr_group<32, 0, CW, PPL, true>), grid, block, 0, st, gp,
                 sp.idx, sp.start, sp.m);
    return hipGetLastError();
  }
  switch (log1 * 2 + (mode ? 1 : 0)) {
#define SLP_GCI(LG, L1)                                                                                            \
  case 2 * LG:                                                                                                    \
    SLP_LAUNCH("col_inv_corr_group_L1_" #L1, (k_colinv_corr_group<L1, 0, CW, PPL>), grid, block, 0, st, gp,   \
               sp.idx, sp.start, sp.m);                                                                           \
    break;                                                                                                        \
  case 2 * LG + 1:                                                                                                \
    SLP_LAUNCH("col_inv_corr_bf16x3_group_L1_" #L1, (k_colinv_corr_group<L1, 1, CW, PPL>), grid, block, 0, st, \
               gp, sp.idx, sp.start, sp.m);                                                                       \
    break;
    SLP_GCI(1, 2) SLP_GCI(2, 4) SLP_GCI(3, 8) SLP_GCI(4, 16) SLP_GCI(5, 32)
#undef SLP_GCI
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t group_colinv_corr(int log1, int mode, int cw, bool one, const GroupPlan *gp, const GroupSpan &sp,
                             hipStream_t st) {
  if (sp.m == 0) return hipSuccess;
  if (cw == 8) return group_colinv_cw<8>(log1, mode, one, gp, sp, st);
  if (cw == 4) return group_colinv_cw<4>(log1, mode, one, gp, sp, st);
  return hipErrorInvalidValue;
}

template hipError_t build_row_tables<float>(const FftGeom &, cpx<float> *, cpx<float> *, hipStream_t);
template hipError_t build_row_tables<double>(const FftGeom &, cpx<double> *, cpx<double> *, hipStream_t);
template hipError_t build_col_table<float>(const FftGeom &, cpx<float> *, hipStream_t);
template hipError_t build_col_table<double>(const FftGeom &, cpx<double> *, hipStream_t);
template hipError_t conv_apply_v2<float>(const float *, int64_t, float *, int64_t, int64_t, int64_t, const FftGeom &,
                                         const FftTables<float> &, float, float, const Corr<float> &, cpx<float> *,
                                         int64_t, hipStream_t);
template hipError_t conv_apply_v2<double>(const double *, int64_t, double *, int64_t, int64_t, int64_t,
                                          const FftGeom &, const FftTables<double> &, double, double,
                                          const Corr<double> &, cpx<double> *, int64_t, hipStream_t);

}  // namespace slp

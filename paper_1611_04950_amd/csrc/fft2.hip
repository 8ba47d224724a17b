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
#include "common.h"
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

// Forward transform, spectrum multiply (spec(z, offset) on each stage-3 job's
// R3 values), inverse transform.  v: lane t's R1 samples x[t + T n1] in,
// L2 * result out.  tw1: the lane's W_L2^{t k1} (k1 < R1), rt2: W_T^{m' k2}
// stored [k2][m'].
template <typename R, int R1, int R2, int R3, typename Spec>
__device__ __forceinline__ void row_conv_core(cpx<R> (&v)[R1], cpx<R> *S, const cpx<R> (&tw1)[R1],
                                              const cpx<R> *__restrict__ rt2, Spec spec) {
  using RS = RowShape<R1, R2, R3>;
  constexpr int T = RS::T;
  const int t = threadIdx.x;
  reg::dft<R1, -1>(v);
#pragma unroll
  for (int k1 = 1; k1 < R1; ++k1) v[k1] = cmul(v[k1], tw1[k1]);
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) S[k1 * RS::S1 + t] = v[k1];
  __syncthreads();
  cpx<R> w[RS::J2][R2];
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
    for (int k2 = 1; k2 < R2; ++k2) w[q][k2] = cmul(w[q][k2], rt2[k2 * R3 + mp]);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) S[k1 * RS::S2K + k2 * RS::S2 + mp] = w[q][k2];
  }
  __syncthreads();
  cpx<R> z[RS::J3][R3];
#pragma unroll
  for (int q = 0; q < RS::J3; ++q) {
    const int g = t + T * q, k2 = g % R2, k1 = g / R2;
#pragma unroll
    for (int m = 0; m < R3; ++m) z[q][m] = S[k1 * RS::S2K + k2 * RS::S2 + m];
    reg::dft<R3, -1>(z[q]);
    spec(z[q], (k1 * R2 + k2) * R3);
    reg::dft<R3, +1>(z[q]);
#pragma unroll
    for (int m = 1; m < R3; ++m) z[q][m] = cmulc(z[q][m], rt2[k2 * R3 + m]);
  }
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

// Middle pass of the three-pass product: row k1c of pair pl, in place.
template <typename R, int R1, int R2, int R3>
__global__ __launch_bounds__(R2 *R3) void k_row2(cpx<R> *__restrict__ Z, int logL, int log2,
                                                 const cpx<R> *__restrict__ rt1, const cpx<R> *__restrict__ rt2,
                                                 const R *__restrict__ chat, R beta, R gl) {
  using RS = RowShape<R1, R2, R3>;
  __shared__ cpx<R> S[RS::LDS];
  const int k1c = blockIdx.x, pl = blockIdx.y;
  cpx<R> *row = Z + ((int64_t)pl << logL) + ((int64_t)k1c << log2);
  const int t = threadIdx.x;
  cpx<R> tw1[R1];
  load_tw1<R, R1, R2, R3>(tw1, rt1);
  cpx<R> v[R1];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) v[n1] = row[t + RS::T * n1];
  const R *ch = chat + ((int64_t)k1c << log2);
  row_conv_core<R, R1, R2, R3>(v, S, tw1, rt2, [&](cpx<R> *z, int off) {
#pragma unroll
    for (int k = 0; k < R3; ++k) z[k] = cscale(z[k], beta * ch[off + k] + gl);
  });
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) row[t + RS::T * n1] = v[n1];
}

// Single-pass product of one signal pair (L = L2).  With CORR the kernel also
// forms C = U^T [x1 x2] (per-lane partial sums, wavefront reductions, a
// fixed-order sum over wavefronts), scales by d, and adds U (d C) to the
// outputs: the whole fast operator of Corollaries 2-4 in one launch.
template <typename R, int R1, int R2, int R3, bool CORR>
__global__ __launch_bounds__(R2 *R3) void k_single2(const R *__restrict__ x, int64_t ldx, R *__restrict__ y,
                                                    int64_t ldy, int N, int b, const cpx<R> *__restrict__ rt1,
                                                    const cpx<R> *__restrict__ rt2, const R *__restrict__ chat,
                                                    R beta, R gl, Corr<R> corr) {
  using RS = RowShape<R1, R2, R3>;
  constexpr int T = RS::T;
  constexpr int NW = T / 64;
  __shared__ cpx<R> S[RS::LDS];
  __shared__ R red[CORR ? NW * kMaxRankSingle * 2 : 2];
  __shared__ R dC[CORR ? 2 * kMaxRankSingle : 2];
  const int t = threadIdx.x;
  const int p = blockIdx.x;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const R *x0 = x + (int64_t)s0 * ldx;
  const R *x1 = x + (int64_t)(has1 ? s1 : s0) * ldx;
  cpx<R> tw1[R1];
  load_tw1<R, R1, R2, R3>(tw1, rt1);
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
  row_conv_core<R, R1, R2, R3>(v, S, tw1, rt2, [&](cpx<R> *z, int off) {
#pragma unroll
    for (int k = 0; k < R3; ++k) z[k] = cscale(z[k], beta * chat[off + k] + gl);
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

// Pass A: lane = column n2 of pair pl; length-L1 DFT of z[n2 + L2 n1] =
// x1 + i x2 (zero for n >= N) in registers, times W_L^{n2 k1}, stored at
// Z[k1][n2].
template <typename R, int L1>
__global__ __launch_bounds__(256) void k_colfwd2(const R *__restrict__ x, int64_t ldx, int N, int b, int pair0,
                                                 int logL, int log2, int s, const cpx<R> *__restrict__ tlo,
                                                 const cpx<R> *__restrict__ thi, cpx<R> *__restrict__ Z) {
  const int n2 = blockIdx.x * 256 + threadIdx.x;
  const int pl = blockIdx.y, p = pair0 + pl;
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
  const int mask = (1 << s) - 1;
  Zp[0] = a[0];
#pragma unroll
  for (int k1 = 1; k1 < L1; ++k1) {
    const int m = n2 * k1;
    Zp[(int64_t)k1 << log2] = cmul(a[k1], cmul(thi[m >> s], tlo[m & mask]));
  }
}

// Pass C: lane = column n2 of pair pl; Z[k1][n2] times W_L^{-n2 k1}, inverse
// length-L1 DFT in registers, y1 = Re and y2 = Im for n = n2 + L2 n1 < N
// (only n1 < L1/2 can hold such n because L >= 2N).
template <typename R, int L1>
__global__ __launch_bounds__(256) void k_colinv2(const cpx<R> *__restrict__ Z, int N, int b, int pair0, int logL,
                                                 int log2, int s, const cpx<R> *__restrict__ tlo,
                                                 const cpx<R> *__restrict__ thi, R *__restrict__ y, int64_t ldy) {
  const int n2 = blockIdx.x * 256 + threadIdx.x;
  const int pl = blockIdx.y, p = pair0 + pl;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const cpx<R> *Zp = Z + ((int64_t)pl << logL) + n2;
  const int mask = (1 << s) - 1;
  cpx<R> a[L1];
  a[0] = Zp[0];
#pragma unroll
  for (int k1 = 1; k1 < L1; ++k1) {
    const int m = n2 * k1;
    a[k1] = cmulc(Zp[(int64_t)k1 << log2], cmul(thi[m >> s], tlo[m & mask]));
  }
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

// Pass C fused with the correction update y += U dC (Corollary 2's U1 U2^T x
// term).  A workgroup of CW wavefronts owns 16 columns c0..c0+15 and 8*CW
// signal pairs; it stages U's rows n = c0 + col + L2 n1 (n1 < L1/2) for all j
// in LDS once.  Lane (col, blk) = (lane % 16, lane / 16) of wavefront w runs the
// inverse column DFTs of pairs 2 blk and 2 blk + 1 of the wavefront's eight
// (one set of twiddles for both), and places the surviving rows straight into
// 16 x 16 matrix-core accumulators D[signal][column] (row 4 blk + v, column
// lane % 16), so the update U dC runs on the matrix cores over j with no
// reshuffle: A = dC^T (signals x j) from memory, B = U^T (j x columns) from LDS.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int L1, int MODE, int CW>
__global__ __launch_bounds__(64 * CW) void k_colinv_corr(const cpx<float> *__restrict__ Z, int N, int b, int pair0,
                                                         int np, int logL, int log2, int s,
                                                         const cpx<float> *__restrict__ tlo,
                                                         const cpx<float> *__restrict__ thi, float *__restrict__ y,
                                                         int64_t ldy, const float *__restrict__ U, int64_t ldu,
                                                         int r, int rp, const float *__restrict__ dC) {
  constexpr int ROWS = L1 > 1 ? L1 / 2 : 1;
  extern __shared__ float Ut[];  // [n1][j][col], ROWS x rp x 16
  const int c0 = blockIdx.x * 16;
  for (int e = threadIdx.x; e < ROWS * rp * 16; e += 64 * CW) {
    const int col = e & 15, j = (e >> 4) % rp, n1 = (e >> 4) / rp;
    const int n = c0 + col + (n1 << log2);
    Ut[e] = (j < r && n < N) ? U[(int64_t)j * ldu + n] : 0.f;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, blk = lane >> 4;
  const int pw = blockIdx.y * 8 * CW + wave * 8;  // first pair of the wavefront, within the slice
  if (pw >= np) return;                            // uniform per wavefront; no barrier follows
  const int n2 = c0 + col;
  const int mask = (1 << s) - 1;
  cpx<float> tw[L1];
#pragma unroll
  for (int k1 = 1; k1 < L1; ++k1) {
    const int m = n2 * k1;
    tw[k1] = cmul(thi[m >> s], tlo[m & mask]);
  }
  f32x4 acc[ROWS];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int pl = pw + 2 * blk + h;
    cpx<float> a[L1];
    if (pl < np) {
      const cpx<float> *Zp = Z + ((int64_t)pl << logL) + n2;
      a[0] = Zp[0];
#pragma unroll
      for (int k1 = 1; k1 < L1; ++k1) a[k1] = cmulc(Zp[(int64_t)k1 << log2], tw[k1]);
    } else {
#pragma unroll
      for (int k1 = 0; k1 < L1; ++k1) a[k1] = cpx<float>{0.f, 0.f};
    }
    reg::dft<L1, +1>(a);
#pragma unroll
    for (int n1 = 0; n1 < ROWS; ++n1) {
      acc[n1][2 * h] = a[n1].x;
      acc[n1][2 * h + 1] = a[n1].y;
    }
  }
  // signals of this wavefront: 2 (pair0 + pw) + 0..15; A row i = lane % 16
  const int sa = 2 * (pair0 + pw) + (lane & 15);
  const bool sav = sa < b && (pw + ((lane & 15) >> 1)) < np;
  const int sac = sav ? sa : 0;
  if constexpr (MODE == 0) {
    for (int jb = 0; jb < rp; jb += 4) {
      const int j = jb + blk;
      const float av = (sav && j < r) ? dC[(int64_t)j * b + sac] : 0.f;
#pragma unroll
      for (int n1 = 0; n1 < ROWS; ++n1)
        acc[n1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Ut[(n1 * rp + j) * 16 + col], acc[n1], 0, 0, 0);
    }
  } else {
    for (int jb = 0; jb < rp; jb += 32) {
      bf16x8 ahi, alo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = jb + 8 * blk + e;
        const float av = (sav && j < r) ? dC[(int64_t)j * b + sac] : 0.f;
        const __bf16 hh = (__bf16)av;
        ahi[e] = hh;
        alo[e] = (__bf16)(av - (float)hh);
      }
#pragma unroll
      for (int n1 = 0; n1 < ROWS; ++n1) {
        bf16x8 bhi, blo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float uv = Ut[(n1 * rp + jb + 8 * blk + e) * 16 + col];
          const __bf16 hh = (__bf16)uv;
          bhi[e] = hh;
          blo[e] = (__bf16)(uv - (float)hh);
        }
        acc[n1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[n1], 0, 0, 0);
        acc[n1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[n1], 0, 0, 0);
        acc[n1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[n1], 0, 0, 0);
      }
    }
  }
  // D[4 blk + v][col] -> signal 2 (pair0 + pw) + 4 blk + v at n = n2 + L2 n1
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int pl = pw + 2 * blk + (v >> 1);
    const int sg = 2 * (pair0 + pw) + 4 * blk + v;
    if (pl >= np || sg >= b) continue;
    float *ys = y + (int64_t)sg * ldy;
#pragma unroll
    for (int n1 = 0; n1 < ROWS; ++n1) {
      const int n = n2 + (n1 << log2);
      if (n < N) ys[n] = acc[n1][v];
    }
  }
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
                       R gl) {
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

template <typename R, int L1>
static void launch_cols(bool fwd, dim3 grid, hipStream_t st, const R *x, int64_t ldx, R *y, int64_t ldy, int N,
                        int b, int p0, const FftGeom &g, const FftTables<R> &tb, cpx<R> *Z) {
  if (fwd) {
    SLP_LAUNCH(sizeof(R) == 4 ? "col_fwd" : "col_fwd_f64", (k_colfwd2<R, L1>), grid, dim3(256), 0, st, x, ldx, N, b,
               p0, g.logL, g.log2, g.s, tb.tw_lo, tb.tw_hi, Z);
  } else {
    SLP_LAUNCH(sizeof(R) == 4 ? "col_inv" : "col_inv_f64", (k_colinv2<R, L1>), grid, dim3(256), 0, st, Z, N, b, p0,
               g.logL, g.log2, g.s, tb.tw_lo, tb.tw_hi, y, ldy);
  }
}

template <typename R>
static bool dispatch_cols(bool fwd, dim3 grid, hipStream_t st, const R *x, int64_t ldx, R *y, int64_t ldy, int N,
                          int b, int p0, const FftGeom &g, const FftTables<R> &tb, cpx<R> *Z) {
  switch (g.log1) {
    case 1: launch_cols<R, 2>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    case 2: launch_cols<R, 4>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    case 3: launch_cols<R, 8>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    case 4: launch_cols<R, 16>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    case 5: launch_cols<R, 32>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    case 6: launch_cols<R, 64>(fwd, grid, st, x, ldx, y, ldy, N, b, p0, g, tb, Z); return true;
    default: return false;
  }
}

constexpr int kColCorrWaves = 4;

int colinv_corr_rp(int r, int mode) { return mode == 0 ? (r + 3) / 4 * 4 : (r + 31) / 32 * 32; }

size_t colinv_corr_lds(int log1, int r, int mode) {
  const int rows = log1 > 0 ? (1 << log1) / 2 : 1;
  return (size_t)rows * colinv_corr_rp(r, mode) * 16 * sizeof(float);
}

template <int L1, int MODE>
static void launch_cic(dim3 grid, size_t lds, hipStream_t st, const cpx<float> *Z, int N, int b, int p0, int np,
                       const FftGeom &g, const FftTables<float> &tb, float *y, int64_t ldy, const Corr<float> &c,
                       int rp) {
  SLP_LAUNCH(MODE ? "col_inv_corr_bf16x3" : "col_inv_corr", (k_colinv_corr<L1, MODE, kColCorrWaves>), grid,
             dim3(64 * kColCorrWaves), lds, st, Z, N, b, p0, np, g.logL, g.log2, g.s, tb.tw_lo, tb.tw_hi, y, ldy, c.U,
             c.ldu, c.r, rp, c.dC);
}

template <int MODE>
static bool launch_cic_mode(hipStream_t st, const cpx<float> *Z, int N, int b, int p0, int np, const FftGeom &g,
                            const FftTables<float> &tb, float *y, int64_t ldy, const Corr<float> &c) {
  const int rp = colinv_corr_rp(c.r, MODE);
  const size_t lds = colinv_corr_lds(g.log1, c.r, MODE);
  const dim3 grid((1u << g.log2) / 16, (unsigned)((np + 8 * kColCorrWaves - 1) / (8 * kColCorrWaves)));
  switch (g.log1) {
    case 1: launch_cic<2, MODE>(grid, lds, st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    case 2: launch_cic<4, MODE>(grid, lds, st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    case 3: launch_cic<8, MODE>(grid, lds, st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    case 4: launch_cic<16, MODE>(grid, lds, st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    case 5: launch_cic<32, MODE>(grid, lds, st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    case 6: launch_cic<64, MODE>(grid, lds, st, Z, N, b, p0, np, g, tb, y, ldy, c, rp); return true;
    default: return false;
  }
}

static bool launch_colinv_corr(hipStream_t st, const cpx<float> *Z, int N, int b, int p0, int np, const FftGeom &g,
                               const FftTables<float> &tb, float *y, int64_t ldy, const Corr<float> &c) {
  return c.mode == 0 ? launch_cic_mode<0>(st, Z, N, b, p0, np, g, tb, y, ldy, c)
                     : launch_cic_mode<1>(st, Z, N, b, p0, np, g, tb, y, ldy, c);
}

#define SLP_ROW_SHAPES(X) \
  X(8, 8, 8)              \
  X(16, 8, 8)             \
  X(16, 16, 8)            \
  X(16, 16, 16)           \
  X(32, 16, 16)

template <typename R>
hipError_t conv_apply_v2(const R *x, int64_t ldx, R *y, int64_t ldy, int64_t N, int64_t b, const FftGeom &g,
                         const FftTables<R> &tb, R beta, R gamma, const Corr<R> &corr, cpx<R> *Z, int64_t slice_pairs,
                         hipStream_t st) {
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
    if (!dispatch_cols<R>(true, gcol, st, x, ldx, y, ldy, (int)N, (int)b, (int)p0, g, tb, Z))
      return hipErrorInvalidValue;
    bool ok = false;
#define SLP_ROW(A, B, C)                                                                                     \
  if (!ok && g.R1 == A && g.R2 == B && g.R3 == C) {                                                           \
    if constexpr (sizeof(R) == 4 || A * B * C <= 4096) {                                                      \
      launch_row<R, A, B, C>(grow, st, Z, g, tb, beta, gl);                                                   \
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

template hipError_t build_row_tables<float>(const FftGeom &, cpx<float> *, cpx<float> *, hipStream_t);
template hipError_t build_row_tables<double>(const FftGeom &, cpx<double> *, cpx<double> *, hipStream_t);
template hipError_t conv_apply_v2<float>(const float *, int64_t, float *, int64_t, int64_t, int64_t, const FftGeom &,
                                         const FftTables<float> &, float, float, const Corr<float> &, cpx<float> *,
                                         int64_t, hipStream_t);
template hipError_t conv_apply_v2<double>(const double *, int64_t, double *, int64_t, int64_t, int64_t,
                                          const FftGeom &, const FftTables<double> &, double, double,
                                          const Corr<double> &, cpx<double> *, int64_t, hipStream_t);

}  // namespace slp

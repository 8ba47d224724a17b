// FFT-based product y = beta * B x + gamma * x (+ optional low-rank correction)
// for gfx950.
//
// B is the N x N prolate (sinc) Toeplitz matrix (Section 1.2, eq. Prolate
// matrix).  Its product with a vector is a linear convolution with the sinc
// sequence, computed as a length-L circular convolution of the zero-padded
// signal with the circulant embedding of B's first column, L the smallest
// power of two >= 2N (Section 1.3 "Fast projections", Section 4.1).  Two real
// signals share one complex transform (x1 + i x2): the embedded kernel is real
// and even, so its spectrum is real and the real and imaginary parts of the
// result are B x1 and B x2 exactly.
//
// Transforms are radix-8/4/2 Stockham passes over LDS: every pass reads its
// operands into registers, synchronises, and writes the butterflies back in
// place, so one LDS buffer serves all passes.  Lengths that fit in one
// workgroup's LDS run as one kernel; longer ones use three passes over a
// workspace (column transforms, row transforms with the spectrum multiply,
// inverse column transforms).
#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

// ---------------------------------------------------------------------------
// Small DFTs in registers.  DIR = -1: forward (exp(-2 pi i nk/R)), +1 inverse.
// ---------------------------------------------------------------------------

template <int DIR, typename R>
__device__ __forceinline__ cpx<R> mul_dir_i(cpx<R> a) {
  return DIR < 0 ? cpx<R>{a.y, -a.x} : cpx<R>{-a.y, a.x};
}

template <int DIR, typename R>
__device__ __forceinline__ void dft2(cpx<R> *a) {
  cpx<R> t = a[0];
  a[0] = t + a[1];
  a[1] = t - a[1];
}

template <int DIR, typename R>
__device__ __forceinline__ void dft4(cpx<R> *a) {
  cpx<R> t0 = a[0] + a[2], t1 = a[0] - a[2];
  cpx<R> t2 = a[1] + a[3], t3 = mul_dir_i<DIR>(a[1] - a[3]);
  a[0] = t0 + t2;
  a[2] = t0 - t2;
  a[1] = t1 + t3;
  a[3] = t1 - t3;
}

template <int DIR, typename R>
__device__ __forceinline__ void dft8(cpx<R> *a) {
  cpx<R> e[4] = {a[0], a[2], a[4], a[6]};
  cpx<R> o[4] = {a[1], a[3], a[5], a[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  const R c = (R)0.70710678118654752440084436210485;
  // w8 = exp(DIR * 2 pi i / 8) = c (1 + DIR i); w8^2 = DIR i; w8^3 = c (-1 + DIR i)
  cpx<R> o1 = {c * (o[1].x - DIR * o[1].y), c * (o[1].y + DIR * o[1].x)};
  cpx<R> o2 = mul_dir_i<DIR>(o[2]);
  cpx<R> o3 = {c * (-o[3].x - DIR * o[3].y), c * (-o[3].y + DIR * o[3].x)};
  a[0] = e[0] + o[0];
  a[4] = e[0] - o[0];
  a[1] = e[1] + o1;
  a[5] = e[1] - o1;
  a[2] = e[2] + o2;
  a[6] = e[2] - o2;
  a[3] = e[3] + o3;
  a[7] = e[3] - o3;
}

template <int DIR, int LOGR, typename R>
__device__ __forceinline__ void dft_r(cpx<R> *a) {
  if constexpr (LOGR == 3) dft8<DIR>(a);
  else if constexpr (LOGR == 2) dft4<DIR>(a);
  else dft2<DIR>(a);
}

// ---------------------------------------------------------------------------
// One Stockham pass over `buf`, laid out [i][c]: transform index i (length
// n = 2^logn) major, batch column c (C = 2^logC) minor.  Job g = (j, c) with
// j in [0, n/R): reads i = j + r n/R, twiddles by W_{Ns R}^{r k} (k = j mod Ns),
// does a radix-R DFT and writes i = (j - k) R + k + r Ns.  After passes with
// Ns = 1, R1, R1 R2, ... the buffer holds the DFT in natural order.
// ---------------------------------------------------------------------------

template <typename R, int DIR, int LOGR, int E>
__device__ __forceinline__ void stockham_pass(cpx<R> *buf, int logn, int logC, int logNs,
                                              const cpx<R> *__restrict__ tw, int logT) {
  constexpr int RAD = 1 << LOGR;
  constexpr int J = (E / RAD + kThreads - 1) / kThreads;
  const int jobs = 1 << (logn - LOGR + logC);
  const int nR = 1 << (logn - LOGR);
  const int Cm = (1 << logC) - 1;
  const int Ns = 1 << logNs;
  cpx<R> v[J][RAD];
#pragma unroll
  for (int q = 0; q < J; ++q) {
    const int g = threadIdx.x + q * kThreads;
    if (g < jobs) {
      const int c = g & Cm, j = g >> logC;
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[q][r] = buf[((j + r * nR) << logC) + c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < J; ++q) {
    const int g = threadIdx.x + q * kThreads;
    if (g < jobs) {
      const int c = g & Cm, j = g >> logC;
      const int k = j & (Ns - 1);
      if (logNs > 0) {
        const int sh = logT - logNs - LOGR;
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          const cpx<R> w = tw[(k * r) << sh];
          v[q][r] = DIR < 0 ? cmul(v[q][r], w) : cmulc(v[q][r], w);
        }
      }
      dft_r<DIR, LOGR>(v[q]);
      const int base = ((j - k) << LOGR) + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[((base + r * Ns) << logC) + c] = v[q][r];
    }
  }
  __syncthreads();
}

// Batched in-place DFT of length 2^logn over 2^logC columns held in LDS.
// tw holds W_T^m = exp(-2 pi i m / T), T = 2^logT >= 2^logn.  Must be called
// by the whole workgroup with uniform arguments.
template <typename R, int DIR, int E>
__device__ void fft_lds(cpx<R> *buf, int logn, int logC, const cpx<R> *__restrict__ tw, int logT) {
  int logNs = 0;
  int rem = logn;
  while (rem > 0) {
    if (rem >= 5 || rem == 3) {
      stockham_pass<R, DIR, 3, E>(buf, logn, logC, logNs, tw, logT);
      logNs += 3;
      rem -= 3;
    } else if (rem == 4 || rem == 2) {
      stockham_pass<R, DIR, 2, E>(buf, logn, logC, logNs, tw, logT);
      logNs += 2;
      rem -= 2;
    } else {
      stockham_pass<R, DIR, 1, E>(buf, logn, logC, logNs, tw, logT);
      logNs += 1;
      rem -= 1;
    }
  }
}

template <typename R>
__device__ __forceinline__ cpx<R> twiddle_L(const FftTables<R> &tb, int s, int m) {
  return cmul(tb.tw_hi[m >> s], tb.tw_lo[m & ((1 << s) - 1)]);
}

// ---------------------------------------------------------------------------
// Single-pass product: one workgroup per signal pair, whole transform in LDS.
// With CORR the workgroup also forms C = U^T [x1 x2] from the signals in LDS
// (one wavefront per column of U), scales it by d, and adds U (d C) to the
// outputs: the fast projection of Corollary 2 in one kernel.
// ---------------------------------------------------------------------------

template <typename R, bool CORR>
__global__ __launch_bounds__(kThreads) void k_conv_single(
    const R *__restrict__ x, int64_t ldx, R *__restrict__ y, int64_t ldy, int N, int b, int logL,
    FftTables<R> tb, int logT, R beta, R gam_over_L, Corr<R> corr) {
  constexpr int E = Lds<R>::E;
  __shared__ cpx<R> buf[E];
  __shared__ R dC[CORR ? 2 * kMaxRankSingle : 2];
  const int L = 1 << logL;
  const int p = blockIdx.x;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const R *x0 = x + (int64_t)s0 * ldx;
  const R *x1 = x + (int64_t)(has1 ? s1 : s0) * ldx;
  for (int n = threadIdx.x; n < L; n += kThreads) {
    R a = 0, c = 0;
    if (n < N) {
      a = x0[n];
      if (has1) c = x1[n];
    }
    buf[n] = cpx<R>{a, c};
  }
  __syncthreads();
  if constexpr (CORR) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = wave; j < corr.r; j += kThreads / 64) {
      const R *u = corr.U + (int64_t)j * corr.ldu;
      R a0 = 0, a1 = 0;
      for (int n = lane; n < N; n += 64) {
        const R uv = u[n];
        const cpx<R> v = buf[n];
        a0 += uv * v.x;
        a1 += uv * v.y;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        a0 += __shfl_xor(a0, off);
        a1 += __shfl_xor(a1, off);
      }
      if (lane == 0) {
        const R dj = corr.d[j];
        dC[2 * j] = dj * a0;
        dC[2 * j + 1] = dj * a1;
      }
    }
  }
  fft_lds<R, -1, E>(buf, logL, 0, tb.tw_sub, logT);
  for (int k = threadIdx.x; k < L; k += kThreads) buf[k] = cscale(buf[k], beta * tb.chat[k] + gam_over_L);
  __syncthreads();
  fft_lds<R, +1, E>(buf, logL, 0, tb.tw_sub, logT);
  R *y0 = y + (int64_t)s0 * ldy;
  R *y1 = y + (int64_t)(has1 ? s1 : s0) * ldy;
  for (int n = threadIdx.x; n < N; n += kThreads) {
    const cpx<R> v = buf[n];
    R a = v.x, c = v.y;
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

// Forward DFT of one real length-L sequence (single pass), complex output in
// natural order.  Used at setup for the kernel spectrum.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_fft_fwd_single(const R *__restrict__ x, int logL,
                                                             cpx<R> *__restrict__ out,
                                                             FftTables<R> tb, int logT) {
  constexpr int E = Lds<R>::E;
  __shared__ cpx<R> buf[E];
  const int L = 1 << logL;
  for (int n = threadIdx.x; n < L; n += kThreads) buf[n] = cpx<R>{x[n], (R)0};
  __syncthreads();
  fft_lds<R, -1, E>(buf, logL, 0, tb.tw_sub, logT);
  for (int k = threadIdx.x; k < L; k += kThreads) out[k] = buf[k];
}

// ---------------------------------------------------------------------------
// Three-pass product.  Workspace Z holds one length-L complex array per pair
// of the current slice, laid out [k1][n2] (rows of length L2).
// ---------------------------------------------------------------------------

// Pass A: for CT consecutive columns n2 of one pair, the length-L1 transforms
// over n1 of z[n2 + L2 n1] = x1 + i x2 (zero for n >= N).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_col_fwd(const R *__restrict__ x, int64_t ldx, int N,
                                                      int b, int pair0, FftGeom g, FftTables<R> tb,
                                                      cpx<R> *__restrict__ Z) {
  constexpr int E = Lds<R>::E;
  __shared__ cpx<R> buf[E];
  const int CTm = (1 << g.logCT) - 1;
  const int c0 = blockIdx.x << g.logCT;
  const int pl = blockIdx.y;
  const int p = pair0 + pl;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const R *x0 = x + (int64_t)s0 * ldx;
  const R *x1 = x + (int64_t)(has1 ? s1 : s0) * ldx;
  const int tile = 1 << (g.log1 + g.logCT);
  for (int e = threadIdx.x; e < tile; e += kThreads) {
    const int i = e >> g.logCT, c = e & CTm;
    const int n = c0 + c + (i << g.log2);
    R a = 0, v = 0;
    if (n < N) {
      a = x0[n];
      if (has1) v = x1[n];
    }
    buf[e] = cpx<R>{a, v};
  }
  __syncthreads();
  fft_lds<R, -1, E>(buf, g.log1, g.logCT, tb.tw_sub, g.logT);
  cpx<R> *Zp = Z + ((int64_t)pl << g.logL);
  for (int e = threadIdx.x; e < tile; e += kThreads) {
    const int k1 = e >> g.logCT, c = e & CTm;
    Zp[((int64_t)k1 << g.log2) + c0 + c] = buf[e];
  }
}

// Pass B: row k1 of one pair.  Twiddle by W_L^{n2 k1}, length-L2 transform
// over n2 (giving X[k1 + L1 k2] at position k2), then either stop (FWD_ONLY,
// setup) or multiply by beta*chat + gamma/L, inverse length-L2 transform, and
// twiddle by W_L^{-n2 k1}.  In place.
template <typename R, bool FWD_ONLY>
__global__ __launch_bounds__(kThreads) void k_row(cpx<R> *__restrict__ Z, FftGeom g, FftTables<R> tb,
                                                  R beta, R gam_over_L) {
  constexpr int E = Lds<R>::E;
  __shared__ cpx<R> buf[E];
  const int L2 = 1 << g.log2;
  const int k1 = blockIdx.x;
  const int pl = blockIdx.y;
  cpx<R> *row = Z + ((int64_t)pl << g.logL) + ((int64_t)k1 << g.log2);
  for (int n2 = threadIdx.x; n2 < L2; n2 += kThreads) buf[n2] = cmul(row[n2], twiddle_L(tb, g.s, n2 * k1));
  __syncthreads();
  fft_lds<R, -1, E>(buf, g.log2, 0, tb.tw_sub, g.logT);
  if constexpr (FWD_ONLY) {
    for (int k2 = threadIdx.x; k2 < L2; k2 += kThreads) row[k2] = buf[k2];
    return;
  } else {
    const R *ch = tb.chat + ((int64_t)k1 << g.log2);
    for (int k2 = threadIdx.x; k2 < L2; k2 += kThreads) buf[k2] = cscale(buf[k2], beta * ch[k2] + gam_over_L);
    __syncthreads();
    fft_lds<R, +1, E>(buf, g.log2, 0, tb.tw_sub, g.logT);
    for (int n2 = threadIdx.x; n2 < L2; n2 += kThreads) row[n2] = cmulc(buf[n2], twiddle_L(tb, g.s, n2 * k1));
  }
}

// Pass C: inverse length-L1 transforms over k1 for CT columns n2 of one pair;
// writes y1 = Re, y2 = Im for n = n2 + L2 n1 < N.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_col_inv(const cpx<R> *__restrict__ Z, FftGeom g,
                                                      FftTables<R> tb, R *__restrict__ y, int64_t ldy,
                                                      int N, int b, int pair0) {
  constexpr int E = Lds<R>::E;
  __shared__ cpx<R> buf[E];
  const int CTm = (1 << g.logCT) - 1;
  const int c0 = blockIdx.x << g.logCT;
  const int pl = blockIdx.y;
  const int p = pair0 + pl;
  const int s0 = 2 * p, s1 = 2 * p + 1;
  const bool has1 = s1 < b;
  const cpx<R> *Zp = Z + ((int64_t)pl << g.logL);
  const int tile = 1 << (g.log1 + g.logCT);
  for (int e = threadIdx.x; e < tile; e += kThreads) {
    const int k1 = e >> g.logCT, c = e & CTm;
    buf[e] = Zp[((int64_t)k1 << g.log2) + c0 + c];
  }
  __syncthreads();
  fft_lds<R, +1, E>(buf, g.log1, g.logCT, tb.tw_sub, g.logT);
  R *y0 = y + (int64_t)s0 * ldy;
  R *y1 = y + (int64_t)(has1 ? s1 : s0) * ldy;
  for (int e = threadIdx.x; e < tile; e += kThreads) {
    const int n1 = e >> g.logCT, c = e & CTm;
    const int n = c0 + c + (n1 << g.log2);
    if (n < N) {
      const cpx<R> v = buf[e];
      y0[n] = v.x;
      if (has1) y1[n] = v.y;
    }
  }
}

// ---------------------------------------------------------------------------
// Setup helpers: twiddle tables, kernel sequence, spectrum layout.
// ---------------------------------------------------------------------------

// out[m] = exp(-2 pi i (m << shift) / 2^logM), m < count, computed in FP64.
template <typename R>
__global__ void k_twiddles(cpx<R> *__restrict__ out, int64_t count, int shift, int logM) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= count) return;
  const double t = ldexp((double)(m << shift), 1 - logM);  // 2 m' / M
  double sn, cs;
  sincospi(t, &sn, &cs);
  out[m] = cpx<R>{(R)cs, (R)(-sn)};
}

// Circulant embedding of B's first column: c[0] = 2W, c[k] = c[L-k] =
// sin(2 pi W k)/(pi k) for 1 <= k <= N-1, zero elsewhere (FP64).
__global__ void k_sinc_embed(double *__restrict__ c, int64_t L, int64_t N, double W) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  int64_t kk = k;
  if (k > L - N) kk = L - k;
  double v = 0.0;
  if (kk == 0) v = 2.0 * W;
  else if (kk < N) v = sinpi(2.0 * W * (double)kk) / (M_PI * (double)kk);
  c[k] = v;
}

// Take the real part / L of a spectrum held in geometry `gs` and store it in
// geometry `gd` (natural index k = k1 + L1 k2 <-> position (k1 << log2) + k2).
template <typename R>
__global__ void k_spectrum_relayout(const cpx<double> *__restrict__ src, FftGeom gs, R *__restrict__ dst,
                                    FftGeom gd) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t L = (int64_t)1 << gs.logL;
  if (pos >= L) return;
  int64_t k;
  if (gs.single()) k = pos;
  else k = (pos >> gs.log2) + ((pos & (((int64_t)1 << gs.log2) - 1)) << gs.log1);
  int64_t pd;
  if (gd.v2) {
    // row k1c = k mod L1; within the row, digits of kr = d1 + R1 d2 + R1 R2 d3
    // stored at (d1 R2 + d2) R3 + d3 (the order the row kernel produces)
    const int64_t k1c = k & (((int64_t)1 << gd.log1) - 1);
    const int64_t kr = k >> gd.log1;
    const int64_t d1 = kr % gd.R1, d2 = (kr / gd.R1) % gd.R2, d3 = kr / ((int64_t)gd.R1 * gd.R2);
    pd = (k1c << gd.log2) + (d1 * gd.R2 + d2) * gd.R3 + d3;
  } else if (gd.single()) {
    pd = k;
  } else {
    pd = ((k & (((int64_t)1 << gd.log1) - 1)) << gd.log2) + (k >> gd.log1);
  }
  dst[pd] = (R)(src[pos].x / (double)L);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

FftGeom make_geom(int logL, int logE, bool allow_v2) {
  FftGeom g;
  g.logL = logL;
  if (logL <= logE) {
    g.log1 = 0;
    g.log2 = logL;
    g.logCT = 0;
    g.logT = logL;
  } else {
    g.log2 = logE;
    g.log1 = logL - logE;
    int lct = logE - g.log1;
    if (lct > 8) lct = 8;
    g.logCT = lct;
    g.logT = g.log1 > g.log2 ? g.log1 : g.log2;
  }
  g.s = (logL + 1) / 2;
  // register-stage rows; columns in registers (L1 <= 32) or through LDS (64..512)
  if (allow_v2 && g.log2 >= 9 && g.log2 <= 13 && g.log1 <= 9) {
    static const int shapes[5][3] = {{8, 8, 8}, {16, 8, 8}, {16, 16, 8}, {16, 16, 16}, {32, 16, 16}};
    const int *sh = shapes[g.log2 - 9];
    g.v2 = 1;
    g.R1 = sh[0];
    g.R2 = sh[1];
    g.R3 = sh[2];
  }
  return g;
}

FftGeom generic_twin(const FftGeom &g) {
  FftGeom t = g;
  t.v2 = 0;
  t.R1 = t.R2 = t.R3 = 0;
  return t;
}

template <typename R>
hipError_t build_tables(const FftGeom &g, cpx<R> *tw_sub, cpx<R> *tw_lo, cpx<R> *tw_hi, hipStream_t st) {
  const int64_t T = (int64_t)1 << g.logT;
  hipLaunchKernelGGL(k_twiddles<R>, dim3((T + 255) / 256), dim3(256), 0, st, tw_sub, T, 0, g.logT);
  if (!g.single()) {
    const int64_t nlo = (int64_t)1 << g.s, nhi = (int64_t)1 << (g.logL - g.s);
    hipLaunchKernelGGL(k_twiddles<R>, dim3((nlo + 255) / 256), dim3(256), 0, st, tw_lo, nlo, 0, g.logL);
    hipLaunchKernelGGL(k_twiddles<R>, dim3((nhi + 255) / 256), dim3(256), 0, st, tw_hi, nhi, g.s, g.logL);
  }
  return hipGetLastError();
}

hipError_t sinc_embed(double *c, int64_t L, int64_t N, double W, hipStream_t st) {
  hipLaunchKernelGGL(k_sinc_embed, dim3((L + 255) / 256), dim3(256), 0, st, c, L, N, W);
  return hipGetLastError();
}

// Forward DFT (FP64) of a real length-L sequence in geometry g; spectrum
// left in `spec` (single: natural order; three-pass: [k1][k2] layout).
hipError_t fft_forward_real64(const double *c, const FftGeom &g, const FftTables<double> &tb,
                              cpx<double> *spec, hipStream_t st) {
  if (g.single()) {
    hipLaunchKernelGGL(k_fft_fwd_single<double>, dim3(1), dim3(kThreads), 0, st, c, g.logL, spec, tb,
                       g.logT);
  } else {
    const int L = 1 << g.logL;
    hipLaunchKernelGGL(k_col_fwd<double>, dim3(1 << (g.log2 - g.logCT), 1), dim3(kThreads), 0, st, c,
                       (int64_t)L, L, 1, 0, g, tb, spec);
    hipLaunchKernelGGL((k_row<double, true>), dim3(1 << g.log1, 1), dim3(kThreads), 0, st, spec, g, tb,
                       0.0, 0.0);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t spectrum_relayout(const cpx<double> *src, const FftGeom &gs, R *dst, const FftGeom &gd,
                             hipStream_t st) {
  const int64_t L = (int64_t)1 << gs.logL;
  hipLaunchKernelGGL(k_spectrum_relayout<R>, dim3((L + 255) / 256), dim3(256), 0, st, src, gs, dst, gd);
  return hipGetLastError();
}

size_t conv_workspace_pairs(const FftGeom &g, int64_t pairs, size_t elem_bytes, size_t budget) {
  if (g.single() || pairs == 0) return 0;
  const size_t per = ((size_t)1 << g.logL) * elem_bytes;
  size_t np = budget / per;
  if (np < 1) np = 1;
  if ((int64_t)np > pairs) np = (size_t)pairs;
  return np;
}

// y = beta B x + gamma x (+ U diag(d) U^T x on the single-pass path when
// corr.r > 0; the three-pass path ignores corr -- the caller applies the
// correction with the separate kernels).  `Z` holds `slice_pairs` pairs.
template <typename R>
hipError_t conv_apply(const R *x, int64_t ldx, R *y, int64_t ldy, int64_t N, int64_t b, const FftGeom &g,
                      const FftTables<R> &tb, R beta, R gamma, const Corr<R> &corr, cpx<R> *Z,
                      int64_t slice_pairs, hipStream_t st) {
  if (g.v2) return conv_apply_v2<R>(x, ldx, y, ldy, N, b, g, tb, beta, gamma, corr, Z, slice_pairs, st);
  const int64_t pairs = (b + 1) / 2;
  if (pairs == 0) return hipSuccess;
  const R gl = gamma / (R)((int64_t)1 << g.logL);
  if (g.single()) {
    for (int64_t p0 = 0; p0 < pairs; p0 += 65535) {
      const int64_t np = pairs - p0 < 65535 ? pairs - p0 : 65535;
      const R *xs = x + 2 * p0 * ldx;
      R *ys = y + 2 * p0 * ldy;
      const int bs = (int)(b - 2 * p0 < 2 * np ? b - 2 * p0 : 2 * np);
      Corr<R> c2 = corr;
      if (corr.r > 0) {
        SLP_LAUNCH("conv_single_corr", (k_conv_single<R, true>), dim3(np), dim3(kThreads), 0, st, xs, ldx, ys, ldy,
                           (int)N, bs, g.logL, tb, g.logT, beta, gl, c2);
      } else {
        SLP_LAUNCH(sizeof(R) == 4 ? "conv_single" : "conv_single_f64", (k_conv_single<R, false>), dim3(np),
                   dim3(kThreads), 0, st, xs, ldx, ys, ldy,
                           (int)N, bs, g.logL, tb, g.logT, beta, gl, c2);
      }
    }
    return hipGetLastError();
  }
  for (int64_t p0 = 0; p0 < pairs; p0 += slice_pairs) {
    const int64_t np = pairs - p0 < slice_pairs ? pairs - p0 : slice_pairs;
    const dim3 gcol(1 << (g.log2 - g.logCT), (unsigned)np);
    const dim3 grow(1 << g.log1, (unsigned)np);
    const bool f = sizeof(R) == 4;
    SLP_LAUNCH(f ? "col_fwd" : "col_fwd_f64", k_col_fwd<R>, gcol, dim3(kThreads), 0, st, x, ldx, (int)N, (int)b,
               (int)p0, g, tb, Z);
    SLP_LAUNCH(f ? "row_conv" : "row_conv_f64", (k_row<R, false>), grow, dim3(kThreads), 0, st, Z, g, tb, beta, gl);
    SLP_LAUNCH(f ? "col_inv" : "col_inv_f64", k_col_inv<R>, gcol, dim3(kThreads), 0, st, Z, g, tb, y, ldy, (int)N,
               (int)b, (int)p0);
  }
  return hipGetLastError();
}

template hipError_t build_tables<float>(const FftGeom &, cpx<float> *, cpx<float> *, cpx<float> *, hipStream_t);
template hipError_t build_tables<double>(const FftGeom &, cpx<double> *, cpx<double> *, cpx<double> *, hipStream_t);
template hipError_t spectrum_relayout<float>(const cpx<double> *, const FftGeom &, float *, const FftGeom &, hipStream_t);
template hipError_t spectrum_relayout<double>(const cpx<double> *, const FftGeom &, double *, const FftGeom &, hipStream_t);
template hipError_t conv_apply<float>(const float *, int64_t, float *, int64_t, int64_t, int64_t, const FftGeom &,
                                      const FftTables<float> &, float, float, const Corr<float> &, cpx<float> *,
                                      int64_t, hipStream_t);
template hipError_t conv_apply<double>(const double *, int64_t, double *, int64_t, int64_t, int64_t, const FftGeom &,
                                       const FftTables<double> &, double, double, const Corr<double> &,
                                       cpx<double> *, int64_t, hipStream_t);

}  // namespace slp

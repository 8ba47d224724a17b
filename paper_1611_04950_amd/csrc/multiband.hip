// Multiband (modulated) Slepian dictionaries (Section 1.4): the projection of
// a real signal onto the union of the Slepian subspaces modulated to band
// centres f_i, each band [f_i - W, f_i + W], approximated by the sum of the
// per-band fast projections
//     y = sum_i w_i Re(E_{f_i} P~ E_{f_i}^* x),   E_f = diag(exp(2 pi i f n)),
// w_i = 2 for f_i > 0 (the band pair +-f_i of a real signal), 1 for f_i = 0.
// Demodulation writes the real and imaginary parts of E_{f_i}^* x_s as two
// adjacent signals, so the product's pair packing transforms them as one
// complex signal (B is real); remodulation takes the real part and sums the
// bands.  Phases are reduced in FP64 (f n mod 1) before the sine and cosine.
//
// Prepared band sets compute the same sum with one FFT product.  For real x,
// Re(E_f B E_f^* x) is the Toeplitz product with the kernel cos(2 pi f m) b(m)
// (B real, symmetric Toeplitz with b(m) = sin(2 pi W m)/(pi m)), so the band
// sum of the B parts is the product with the single real symmetric Toeplitz
// kernel b(m) sum_i w_i cos(2 pi f_i m), whose circulant spectrum is computed
// once.  The correction parts, with m_{i,0}(n) = cos(2 pi f_i n) and
// m_{i,1}(n) = -sin(2 pi f_i n), are
//     sum_i w_i sum_c (m_{i,c} (.) U) diag(d) (m_{i,c} (.) U)^T x,
// a correction of rank 2 J r whose modulated columns are formed in registers
// from U and a table of the m_{i,c} (prepared once per band set, FP32 from
// FP64 phases): C'[j][(i,c,s)] = sum_n U[n][j] m_{i,c}(n) x_s(n) on the
// matrix cores in 32 x 32 tiles, weights w_i d_j, then
//     y_s(n) += sum_(i,c) m_{i,c}(n) sum_j U[n][j] dC'[j][(i,c,s)]
// in 16 x 16 tiles (signals x samples), one matrix-core product per (i, c)
// scaled by the sample's m_{i,c}(n).  The table carries one extra zero row,
// which lanes without a modulation read, so that no load is conditional.
// The table and U's copy for the coefficients are stored in blocks of 8
// samples ([n / 8][row][8]): the rows a wavefront reads for one step are then
// one contiguous segment instead of rows megabytes apart.
#include <cstdlib>

#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

__device__ __forceinline__ void band_phase(double f, int64_t n, double &c, double &s) {
  const double t = f * (double)n;
  const double fr = t - floor(t);  // f n mod 1
  sincospi(2.0 * fr, &s, &c);
}

// z[2 (i b + s)][n] = x_s[n] cos(2 pi f_i n), z[2 (i b + s) + 1][n] = -x_s[n] sin(2 pi f_i n)
__global__ __launch_bounds__(256) void k_demod(const float *__restrict__ x, int64_t ldx, int N, int b, BandSet bs,
                                               float *__restrict__ z, int64_t ldz) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y, i = blockIdx.z;
  if (n >= N) return;
  double c, sn;
  band_phase(bs.f[i], n, c, sn);
  const double v = x[(int64_t)s * ldx + n];
  const int64_t q = 2 * ((int64_t)i * b + s);
  z[q * ldz + n] = (float)(v * c);
  z[(q + 1) * ldz + n] = (float)(-v * sn);
}

// y_s[n] = sum_i w_i (cos(2 pi f_i n) p[2 (i b + s)][n] - sin(2 pi f_i n) p[2 (i b + s) + 1][n])
__global__ __launch_bounds__(256) void k_remod(const float *__restrict__ p, int64_t ldp, int N, int b, BandSet bs,
                                               float *__restrict__ y, int64_t ldy) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (n >= N) return;
  double acc = 0.0;
  for (int i = 0; i < bs.J; ++i) {
    double c, sn;
    band_phase(bs.f[i], n, c, sn);
    const int64_t q = 2 * ((int64_t)i * b + s);
    const double w = bs.f[i] > 0.0 ? 2.0 : 1.0;
    acc += w * (c * (double)p[q * ldp + n] - sn * (double)p[(q + 1) * ldp + n]);
  }
  y[(int64_t)s * ldy + n] = (float)acc;
}

hipError_t band_demod(const float *x, int64_t ldx, int64_t N, int64_t b, const BandSet &bs, float *z, int64_t ldz,
                      hipStream_t st) {
  if (N == 0 || b == 0 || bs.J == 0) return hipSuccess;
  if (b > 65535 || bs.J > kMaxBands) return hipErrorInvalidValue;
  SLP_LAUNCH("band_demod", k_demod, dim3((unsigned)((N + 255) / 256), (unsigned)b, (unsigned)bs.J), dim3(256), 0, st,
             x, ldx, (int)N, (int)b, bs, z, ldz);
  return hipGetLastError();
}

hipError_t band_remod(const float *p, int64_t ldp, int64_t N, int64_t b, const BandSet &bs, float *y, int64_t ldy,
                      hipStream_t st) {
  if (N == 0 || b == 0) return hipSuccess;
  if (b > 65535 || bs.J > kMaxBands) return hipErrorInvalidValue;
  SLP_LAUNCH("band_remod", k_remod, dim3((unsigned)((N + 255) / 256), (unsigned)b), dim3(256), 0, st, p, ldp,
             (int)N, (int)b, bs, y, ldy);
  return hipGetLastError();
}

// ---- prepared band sets ----

// Circulant embedding (length L) of the band-sum kernel
// k(m) = b(m) sum_i w_i cos(2 pi f_i m), |m| <= N - 1, zero elsewhere (FP64).
__global__ __launch_bounds__(256) void k_band_embed(double *__restrict__ c, int64_t L, int64_t N, double W,
                                                    BandSet bs) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= L) return;
  const int64_t m = k > L - N ? L - k : k;
  double v = 0.0;
  if (m < N) {
    const double bm = m == 0 ? 2.0 * W : sinpi(2.0 * W * (double)m) / (M_PI * (double)m);
    double sum = 0.0;
    for (int i = 0; i < bs.J; ++i) {
      double cs, sn;
      band_phase(bs.f[i], m, cs, sn);
      sum += (bs.f[i] > 0.0 ? 2.0 : 1.0) * cs;
    }
    v = bm * sum;
  }
  c[k] = v;
}

// Blocked table: M[((n / 8) (2J + 1) + 2 i + c) 8 + n % 8] = m_{i,c}(n) for
// n < N, zero for N <= n < ldm; row 2J is all zero.  Grid (ldm / 256, J + 1).
__global__ __launch_bounds__(256) void k_band_table(float *__restrict__ M, int64_t ldm, int N, BandSet bs) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  if (n >= ldm) return;
  const int64_t base = ((n >> 3) * (2 * bs.J + 1)) * 8 + (n & 7);
  if (i == bs.J) {
    M[base + (int64_t)(2 * i) * 8] = 0.f;
    return;
  }
  float c = 0.f, s = 0.f;
  if (n < N) {
    double cd, sd;
    band_phase(bs.f[i], n, cd, sd);
    c = (float)cd;
    s = (float)(-sd);
  }
  M[base + (int64_t)(2 * i) * 8] = c;
  M[base + (int64_t)(2 * i + 1) * 8] = s;
}

hipError_t band_embed(double *c, int64_t L, int64_t N, double W, const BandSet &bs, hipStream_t st) {
  SLP_LAUNCH("band_embed", k_band_embed, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, st, c, L, N, W, bs);
  return hipGetLastError();
}

int64_t band_table_rows(int J) { return 2 * (int64_t)J + 1; }

int64_t mb_ldm(int64_t N) { return (N + 63) / 64 * 64; }

hipError_t band_table(float *M, int64_t ldm, int64_t N, const BandSet &bs, hipStream_t st) {
  if (ldm < N || ldm % 64 != 0 || bs.J < 1 || bs.J > kMaxBands) return hipErrorInvalidValue;
  SLP_LAUNCH("band_table", k_band_table, dim3((unsigned)((ldm + 255) / 256), (unsigned)(bs.J + 1)), dim3(256), 0,
             st, M, ldm, (int)N, bs);
  return hipGetLastError();
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// v = hi + lo with hi = bf16(v) and lo = bf16(v - hi), two values per conversion
__device__ __forceinline__ void mb_split(const float (&v)[8], bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const f32x2 a = {v[2 * p], v[2 * p + 1]};
    const bf16x2 h = __builtin_convertvector(a, bf16x2);
    const bf16x2 l = __builtin_convertvector(a - __builtin_convertvector(h, f32x2), bf16x2);
    hi[2 * p] = h[0];
    hi[2 * p + 1] = h[1];
    lo[2 * p] = l[0];
    lo[2 * p + 1] = l[1];
  }
}

template <bool VEC>
__device__ __forceinline__ void mb_load8(const float *__restrict__ p, float (&v)[8]) {
  if constexpr (VEC) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    const float4 c = *reinterpret_cast<const float4 *>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = p[e];
  }
}

// U's columns laid out for the modulated correction, built once per plan: a
// blocked copy Ub[((n / 8) rpad + j) 8 + n % 8] (rpad = 32 ceil(r / 32) rows,
// n < ldm, zero for j >= r or n >= N) for the coefficients, as BF16 hi/lo
// planes (Uh, Ul) or FP32 (U32b), and U^T planes [n][jp] (j fastest, zero for
// j >= r) in BF16 hi/lo (Th, Tl) or FP32 (T32) for the update.
__global__ __launch_bounds__(256) void k_mb_ublock(const float *__restrict__ U, int64_t ldu, int N, int r, int rpad,
                                                   int64_t ldm, __bf16 *__restrict__ Uh, __bf16 *__restrict__ Ul,
                                                   float *__restrict__ U32b) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (n >= ldm) return;
  const float v = (j < r && n < N) ? U[(int64_t)j * ldu + n] : 0.f;
  const int64_t o = ((n >> 3) * rpad + j) * 8 + (n & 7);
  if (U32b) {
    U32b[o] = v;
  } else {
    const __bf16 h = (__bf16)v;
    Uh[o] = h;
    Ul[o] = (__bf16)(v - (float)h);
  }
}

__global__ __launch_bounds__(256) void k_mb_utrans(const float *__restrict__ U, int64_t ldu, int N, int r, int jp,
                                                   __bf16 *__restrict__ Th, __bf16 *__restrict__ Tl,
                                                   float *__restrict__ T32) {
  __shared__ float tile[32][65];
  const int n0 = blockIdx.x * 64, j0 = blockIdx.y * 32;
  for (int e = threadIdx.x; e < 32 * 64; e += 256) {
    const int jj = e >> 6, nn = e & 63;
    const int j = j0 + jj, n = n0 + nn;
    tile[jj][nn] = (j < r && n < N) ? U[(int64_t)j * ldu + n] : 0.f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 64; e += 256) {
    const int nn = e >> 5, jj = e & 31;
    const int n = n0 + nn;
    if (n >= N) continue;
    const float v = tile[jj][nn];
    const int64_t o = (int64_t)n * jp + j0 + jj;
    if (T32) T32[o] = v;
    if (Th) {
      const __bf16 h = (__bf16)v;
      Th[o] = h;
      Tl[o] = (__bf16)(v - (float)h);
    }
  }
}

hipError_t mb_ulayout(int mode, const float *U, int64_t ldu, int64_t N, int r, int64_t ldm, __bf16 *Uh, __bf16 *Ul,
                      float *U32b, __bf16 *Th, __bf16 *Tl, float *T32, hipStream_t st) {
  if (r <= 0 || r > kMbMaxRank || ldm < N || ldm % 64 != 0) return hipErrorInvalidValue;
  const int rpad = (r + 31) / 32 * 32;
  SLP_LAUNCH("mb_ublock", k_mb_ublock, dim3((unsigned)((ldm + 255) / 256), (unsigned)rpad), dim3(256), 0, st, U, ldu,
             (int)N, r, rpad, ldm, Uh, Ul, mode != 0 ? nullptr : U32b);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SLP_LAUNCH("mb_utrans", k_mb_utrans, dim3((unsigned)((N + 63) / 64), (unsigned)(rpad / 32)), dim3(256), 0, st, U,
             ldu, (int)N, r, rpad, mode != 0 ? Th : nullptr, mode != 0 ? Tl : nullptr, mode != 0 ? nullptr : T32);
  return hipGetLastError();
}

// C' partials.  Workgroup = nw (up to 4) wavefronts on one chunk of 32 * steps
// samples (blockIdx.x); wavefront w holds NBW 32 x 32 accumulators, the column
// blocks (nw cg + w) NBW + nb of the 32-column blocks of C'.  Rows are
// j = 32 blockIdx.z + lane % 32 (U columns); columns are packed as G = 2^logG
// signals times 32 / G modulations, so lane i serves signal s = G sg + i % G
// (the same in every accumulator) and modulation cmb = blk 32/G + i / G
// (blockIdx.y = cg nsg + sg).  The chunk is processed in stages of SS samples:
// the workgroup first copies the R = nw NBW 32/G table rows of its
// modulations (rows past the last one read the table's zero row) and its G
// signals for the stage into LDS with coalesced loads, then every wavefront
// reads its operands from LDS, where lanes that share a value are served by
// one broadcast.  U comes from its blocked copy (BF16 hi/lo for MODE 1, FP32
// for MODE 0; zero rows past r, zero beyond N).  Lanes past the last signal or
// U column compute columns and rows that are never stored.  Each wavefront
// stores its own columns of the chunk's partial,
// part[(chunk rpad + j) ncol + cmb b + s].
template <int MODE, int NBW, bool VEC>
__global__ __launch_bounds__(256) void k_mb_partial(const float *__restrict__ X, int64_t ldx, int N, int b,
                                                    const float *__restrict__ U32b, const __bf16 *__restrict__ Uh,
                                                    const __bf16 *__restrict__ Ul, int r,
                                                    const float *__restrict__ M, int ncmb, int logG, int nsg, int nw,
                                                    int steps, int SS, float *__restrict__ part, int rpad) {
  extern __shared__ float lds[];
  const int nthr = 64 * nw;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 31, kb = lane >> 5;
  const int G = 1 << logG, cpb = 32 >> logG;
  const int sg = blockIdx.y % nsg, cg = blockIdx.y / nsg;
  const int R = nw * NBW * cpb;        // table rows staged by this workgroup
  const int cmb0 = cg * R;             // its first modulation
  const int blk0 = (cg * nw + wave) * NBW;
  const bool active = blk0 * cpb < ncmb;  // wave-uniform
  const int XS = SS + 4;               // padded LDS row of a signal
  float *tabL = lds;                   // [SS / 8][R][8]
  float *xL = lds + SS * R;            // [G][XS]
  const int s = sg * G + (i & (G - 1));
  const bool sv = s < b;
  const int j = blockIdx.z * 32 + i;  // < rpad
  const int mrows = ncmb + 1;
  int rl[NBW];
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) rl[nb] = (wave * NBW + nb) * cpb + (i >> logG);  // row within tabL
  f32x16 acc[NBW];
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[nb][v] = 0.f;
  const int k_begin = blockIdx.x * steps * 32;
  const int k_end = min(N, k_begin + steps * 32);
  for (int st0 = k_begin; st0 < k_end; st0 += SS) {
    __syncthreads();  // the previous stage has been read
    // stage the table rows: (SS / 8) blocks x R rows x two float4
    const int tunits = (SS / 8) * R * 2;
    for (int u = threadIdx.x; u < tunits; u += nthr) {
      const int n8 = u / (2 * R), rem = u - n8 * 2 * R, row = rem >> 1, half = rem & 1;
      const int g = min(cmb0 + row, ncmb);
      // blocks at or past N lie beyond the table's padded length for the last stage: zero
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (st0 + 8 * n8 < N) v = *reinterpret_cast<const float4 *>(M + (((int64_t)(st0 >> 3) + n8) * mrows + g) * 8 + 4 * half);
      *reinterpret_cast<float4 *>(tabL + (n8 * R + row) * 8 + 4 * half) = v;
    }
    // stage the signals: G rows x SS samples (zero beyond N)
    const int xunits = G * (SS / 4);
    for (int u = threadIdx.x; u < xunits; u += nthr) {
      const int row = u / (SS / 4), c4 = u - row * (SS / 4);
      const int sr = min(sg * G + row, b - 1);
      const int n = st0 + 4 * c4;
      const float *xp = X + (int64_t)sr * ldx + n;
      float4 v;
      if (VEC && n + 4 <= N) {
        v = *reinterpret_cast<const float4 *>(xp);
      } else {
        v.x = n < N ? xp[0] : 0.f;
        v.y = n + 1 < N ? xp[1] : 0.f;
        v.z = n + 2 < N ? xp[2] : 0.f;
        v.w = n + 3 < N ? xp[3] : 0.f;
      }
      *reinterpret_cast<float4 *>(xL + row * XS + 4 * c4) = v;
    }
    __syncthreads();
    if (active) {
      const int st1 = min(k_end, st0 + SS);
      for (int k0 = st0; k0 < st1; k0 += 32) {
        const int kl = k0 - st0;
        float ua[MODE == 0 ? 2 : 1][8], xv[2][8];
        bf16x8 ah[2], al[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int kk = k0 + 16 * q + 8 * kb;
          // the blocked copies are zero-padded to ldm >= N rounded up to 64: no guard
          const int64_t ub = ((int64_t)(kk >> 3) * rpad + j) * 8;
          if constexpr (MODE == 0) {
            mb_load8<true>(U32b + ub, ua[q]);
          } else {
            ah[q] = *reinterpret_cast<const bf16x8 *>(Uh + ub);
            al[q] = *reinterpret_cast<const bf16x8 *>(Ul + ub);
          }
          const float *xr = xL + (i & (G - 1)) * XS + kl + 16 * q + 8 * kb;
          const float4 x0 = *reinterpret_cast<const float4 *>(xr);
          const float4 x1 = *reinterpret_cast<const float4 *>(xr + 4);
          xv[q][0] = x0.x; xv[q][1] = x0.y; xv[q][2] = x0.z; xv[q][3] = x0.w;
          xv[q][4] = x1.x; xv[q][5] = x1.y; xv[q][6] = x1.z; xv[q][7] = x1.w;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int n8 = (kl + 16 * q + 8 * kb) >> 3;
#pragma unroll
          for (int nb = 0; nb < NBW; ++nb) {
            const float *mr = tabL + (n8 * R + rl[nb]) * 8;
            const float4 m0 = *reinterpret_cast<const float4 *>(mr);
            const float4 m1 = *reinterpret_cast<const float4 *>(mr + 4);
            float bv[8];
            bv[0] = xv[q][0] * m0.x; bv[1] = xv[q][1] * m0.y; bv[2] = xv[q][2] * m0.z; bv[3] = xv[q][3] * m0.w;
            bv[4] = xv[q][4] * m1.x; bv[5] = xv[q][5] * m1.y; bv[6] = xv[q][6] * m1.z; bv[7] = xv[q][7] * m1.w;
            if constexpr (MODE == 0) {
#pragma unroll
              for (int e = 0; e < 8; ++e)
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ua[q][e], bv[e], acc[nb], 0, 0, 0);
            } else {
              bf16x8 bhi, blo;
              mb_split(bv, bhi, blo);
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[q], bhi, acc[nb], 0, 0, 0);
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[q], blo, acc[nb], 0, 0, 0);
              acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[q], bhi, acc[nb], 0, 0, 0);
            }
          }
        }
      }
    }
  }
  if (!active || !sv) return;
  const int ncol = ncmb * b;
  float *pc = part + (int64_t)blockIdx.x * rpad * ncol;
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) {
    const int cmb = (blk0 + nb) * cpb + (i >> logG);
    if (cmb >= ncmb) continue;
    const int col = cmb * b + s;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int jj = blockIdx.z * 32 + 8 * (v >> 2) + 4 * kb + (v & 3);
      if (jj < r) pc[(int64_t)jj * ncol + col] = acc[nb][v];
    }
  }
}

// dC'[col jp + j] = w_band d_j sum over chunks of part[(chunk rpad + j) ncol + col]
// (zero for r <= j < jp), with its BF16 hi/lo planes H and Lo in the same
// layout; col = cmb b + s, band = cmb / 2.  16 outputs per workgroup
// (consecutive col), 16 lanes per output each summing every 16th chunk, then a
// fixed-order sum of the 16 through LDS.
__global__ __launch_bounds__(256) void k_mb_reduce(const float *__restrict__ part, int chunks, int rpad, int ncol,
                                                   int b, int r, int jp, const float *__restrict__ d,
                                                   float *__restrict__ D, __bf16 *__restrict__ H,
                                                   __bf16 *__restrict__ Lo, BandSet bs) {
  __shared__ float red[16][17];
  const int og = threadIdx.x & 15, cgp = threadIdx.x >> 4;
  const int64_t o = (int64_t)blockIdx.x * 16 + og;  // o = j ncol + col
  const bool valid = o < (int64_t)jp * ncol;
  const int j = valid ? (int)(o / ncol) : 0, col = valid ? (int)(o % ncol) : 0;
  float acc = 0.f;
  if (valid && j < r) {
    const int64_t stride = (int64_t)rpad * ncol;
    const float *pp = part + (int64_t)j * ncol + col;
    for (int c0 = cgp; c0 < chunks; c0 += 128) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = c0 + 16 * e;
        v[e] = c < chunks ? pp[(int64_t)c * stride] : 0.f;
      }
      acc += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
  }
  red[cgp][og] = acc;
  __syncthreads();
  if (cgp == 0 && valid) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][og];
    const int band = (col / b) >> 1;
    const float v = j < r ? (bs.f[band] > 0.0 ? 2.f : 1.f) * (d[j] * t) : 0.f;
    const int64_t od = (int64_t)col * jp + j;
    D[od] = v;
    const __bf16 h = (__bf16)v;
    H[od] = h;
    Lo[od] = (__bf16)(v - (float)h);
  }
}

// y += the modulated update.  A wavefront owns 16 signals (s0 = 16 blockIdx.y)
// and T consecutive 16-sample tiles; lane (c, q) = (lane % 16, lane / 16);
// the workgroup's 4 wavefronts cover 64 T consecutive samples.  The table
// rows of up to 64 / T modulations at a time are first copied into LDS
// (coalesced, zero past N and past the last modulation).  A = dC'^T (row c:
// signal s0 + c; k: j) is loaded for CU modulations at a time and reused for
// the T tiles; B = U^T (k: j; column c: sample n0 + 16 t + c) comes from the
// plan's [n][jp] layout of U, one vector load per 8 (BF16) or 4 (FP32)
// consecutive j, once per tile.  Per modulation and tile, a product over j
// into tt, then acc += m_cmb(n) tt.  D[4 q + v][c] is signal s0 + 4 q + v at
// the sample of column c.  Lanes past the last signal read a clamped row of
// dC' and are not stored.
template <int MODE, int RK, int T, int CU>
__global__ __launch_bounds__(256) void k_mb_apply(float *__restrict__ Y, int64_t ldy, int N, int b,
                                                  const float *__restrict__ T32, const __bf16 *__restrict__ Th,
                                                  const __bf16 *__restrict__ Tl, const float *__restrict__ M,
                                                  int ncmb, const float *__restrict__ D,
                                                  const __bf16 *__restrict__ H, const __bf16 *__restrict__ Lo) {
  constexpr int JP = 32 * RK;
  constexpr int WS = 64 * T;        // samples per workgroup
  constexpr int CCM = 4096 / WS;    // modulations per LDS stage (a multiple of CU)
  __shared__ float tabA[WS / 8][CCM][8];
  const int lane = threadIdx.x & 63, c = lane & 15, q = lane >> 4, wave = threadIdx.x >> 6;
  const int nW = blockIdx.x * WS;
  const int n0 = nW + wave * 16 * T;
  const bool active = n0 < N;  // wave-uniform
  const int s0 = blockIdx.y * 16;
  const int sa = s0 + c;
  const int sac = sa < b ? sa : b - 1;
  const int mrows = ncmb + 1;
  int nc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int n = n0 + 16 * t + c;
    nc[t] = n < N ? n : N - 1;
  }
  // B operand: U[j][n] for this lane's j, every tile
  float4 uf[MODE == 0 ? T : 1][MODE == 0 ? JP / 16 : 1];
  bf16x8 uh[MODE == 0 ? 1 : T][MODE == 0 ? 1 : RK], ul[MODE == 0 ? 1 : T][MODE == 0 ? 1 : RK];
  f32x4 acc[T];
  if (active) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int64_t row = (int64_t)nc[t] * JP;
      if constexpr (MODE == 0) {
#pragma unroll
        for (int g = 0; g < JP / 16; ++g) uf[t][g] = *reinterpret_cast<const float4 *>(T32 + row + 16 * g + 4 * q);
      } else {
#pragma unroll
        for (int k = 0; k < RK; ++k) {
          uh[t][k] = *reinterpret_cast<const bf16x8 *>(Th + row + 32 * k + 8 * q);
          ul[t][k] = *reinterpret_cast<const bf16x8 *>(Tl + row + 32 * k + 8 * q);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int sg = s0 + 4 * q + v;
        const int n = n0 + 16 * t + c;
        acc[t][v] = (sg < b && n < N) ? Y[(int64_t)sg * ldy + n] : 0.f;
      }
  }
  for (int c0 = 0; c0 < ncmb; c0 += CCM) {
    __syncthreads();  // the previous stage has been read
    for (int u = threadIdx.x; u < (WS / 8) * CCM * 2; u += 256) {
      const int n8 = u / (2 * CCM), rem = u - n8 * 2 * CCM, row = rem >> 1, half = rem & 1;
      const int cmb = c0 + row;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (cmb < ncmb && nW + 8 * n8 < N)
        v = *reinterpret_cast<const float4 *>(M + (((int64_t)(nW >> 3) + n8) * mrows + cmb) * 8 + 4 * half);
      *reinterpret_cast<float4 *>(&tabA[n8][row][4 * half]) = v;
    }
    __syncthreads();
    if (!active) continue;
    const int c1 = min(ncmb, c0 + CCM);
    for (int cb = c0; cb < c1; cb += CU) {
      float mv[CU][T];
#pragma unroll
      for (int u = 0; u < CU; ++u)
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int nl = wave * 16 * T + 16 * t + c;
          mv[u][t] = tabA[nl >> 3][cb - c0 + u][nl & 7];  // zero past the last modulation
        }
      if constexpr (MODE == 0) {
        float4 a[CU][JP / 16];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
          const int cmb = cb + u < ncmb ? cb + u : ncmb - 1;
          const int64_t arow = ((int64_t)cmb * b + sac) * JP;
#pragma unroll
          for (int g = 0; g < JP / 16; ++g) a[u][g] = *reinterpret_cast<const float4 *>(D + arow + 16 * g + 4 * q);
        }
#pragma unroll
        for (int u = 0; u < CU; ++u)
#pragma unroll
          for (int t = 0; t < T; ++t) {
            f32x4 tt = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int g = 0; g < JP / 16; ++g) {
              tt = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][g].x, uf[t][g].x, tt, 0, 0, 0);
              tt = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][g].y, uf[t][g].y, tt, 0, 0, 0);
              tt = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][g].z, uf[t][g].z, tt, 0, 0, 0);
              tt = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][g].w, uf[t][g].w, tt, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][v] += mv[u][t] * tt[v];
          }
      } else {
        bf16x8 ah[CU][RK], al[CU][RK];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
          const int cmb = cb + u < ncmb ? cb + u : ncmb - 1;
          const int64_t arow = ((int64_t)cmb * b + sac) * JP;
#pragma unroll
          for (int k = 0; k < RK; ++k) {
            ah[u][k] = *reinterpret_cast<const bf16x8 *>(H + arow + 32 * k + 8 * q);
            al[u][k] = *reinterpret_cast<const bf16x8 *>(Lo + arow + 32 * k + 8 * q);
          }
        }
#pragma unroll
        for (int u = 0; u < CU; ++u)
#pragma unroll
          for (int t = 0; t < T; ++t) {
            f32x4 tt = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < RK; ++k) {
              tt = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u][k], uh[t][k], tt, 0, 0, 0);
              tt = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u][k], ul[t][k], tt, 0, 0, 0);
              tt = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[u][k], uh[t][k], tt, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][v] += mv[u][t] * tt[v];
          }
      }
    }
  }
  if (!active) return;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int n = n0 + 16 * t + c;
    if (n >= N) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int sg = s0 + 4 * q + v;
      if (sg < b) Y[(int64_t)sg * ldy + n] = acc[t][v];
    }
  }
}

static int mb_logG(int64_t b) {
  int lg = 0;
  while (lg < 5 && ((int64_t)1 << lg) < b) ++lg;
  return lg;
}

static int env_int(const char *name, int dflt) {
  const char *e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}

// tuning overrides, read once per process
struct MbTuning {
  int nbw1, pwaves, tiles, cu;
  MbTuning()
      : nbw1(env_int("SLEPIAN_MB_NBW", 0) == 1), pwaves(env_int("SLEPIAN_MB_PWAVES", 4096)),
        tiles(env_int("SLEPIAN_MB_T", 4)), cu(env_int("SLEPIAN_MB_CU", 4)) {}
};
static const MbTuning &mb_tuning() {
  static const MbTuning t;
  return t;
}

MbShape mb_shape(int64_t N, int64_t b, int r, int J) {
  MbShape sh;
  sh.ncmb = 2 * J;
  sh.logG = mb_logG(b);
  const int G = 1 << sh.logG, cpb = 32 / G;
  sh.nsg = (int)((b + G - 1) / G);
  const int nblk = (sh.ncmb + cpb - 1) / cpb;
  sh.nbw = nblk >= 8 ? 2 : 1;
  if (mb_tuning().nbw1) sh.nbw = 1;  // tuning override
  const int per = (nblk + sh.nbw - 1) / sh.nbw;  // wavefronts needed for all blocks
  sh.nw = per < 4 ? per : 4;
  sh.ncg = (nblk + sh.nw * sh.nbw - 1) / (sh.nw * sh.nbw);
  sh.nz = (r + 31) / 32;
  sh.rpad = 32 * sh.nz;
  sh.jp = 32 * sh.nz;
  // about 4096 wavefronts in the partial pass (tuning override SLEPIAN_MB_PWAVES)
  int64_t waves = mb_tuning().pwaves;
  if (waves < 256 || waves > 65536) waves = 4096;
  const int64_t per_chunk = (int64_t)sh.nw * sh.ncg * sh.nsg * sh.nz;
  const int64_t want = per_chunk >= waves ? 1 : waves / per_chunk;
  int64_t steps = (N + 32 * want - 1) / (32 * want);
  if (steps < 1) steps = 1;
  if (steps > 1024) steps = 1024;
  // LDS stage: R table rows and G signal rows of SS samples, SS R <= 4096 floats
  const int R = sh.nw * sh.nbw * cpb;
  int ss = 256;
  while (ss > 32 && ss * R > 4096) ss >>= 1;
  sh.ss = ss;
  if (steps % (ss / 32) != 0) steps = (steps + ss / 32 - 1) / (ss / 32) * (ss / 32);
  sh.lds_bytes = (ss * R + G * (ss + 4)) * (int)sizeof(float);
  sh.steps = (int)steps;
  sh.chunks = (int)((N + 32 * steps - 1) / (32 * steps));
  // apply: 16-sample tiles per wavefront and modulations per iteration
  // (tuning overrides SLEPIAN_MB_T, SLEPIAN_MB_CU for one 32-row block)
  const int rk = sh.nz;
  sh.tiles = rk == 1 ? 4 : (rk == 2 ? 4 : 2);
  sh.cu = rk == 1 ? 4 : 1;
  if (rk == 1) {
    const int t = mb_tuning().tiles, cu = mb_tuning().cu;
    if (t == 4 || t == 8) sh.tiles = t;
    if (cu == 1 || cu == 4) sh.cu = cu;
  }
  return sh;
}

bool mb_ok(const MbShape &sh, int64_t N, int64_t b, int r) {
  const int64_t ncol = (int64_t)sh.ncmb * b;
  return r <= kMbMaxRank && N < ((int64_t)1 << 31) - 32 * 1024 && (int64_t)sh.nsg * sh.ncg <= 65535 &&
         (b + 15) / 16 <= 65535 && ncol <= 0x7fffffff && (ncol * sh.jp + 15) / 16 <= 0x7fffffff;
}

size_t mb_workspace_bytes(const MbShape &sh, int64_t b) {
  const size_t ncol = (size_t)sh.ncmb * b;
  const size_t part = (size_t)sh.chunks * sh.rpad * ncol * sizeof(float);
  const size_t dc = ncol * sh.jp;
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  return al(part) + al(dc * sizeof(float)) + 2 * al(dc * sizeof(__bf16));
}

MbWs mb_carve(const MbShape &sh, int64_t b, void *ws) {
  const int64_t ncol = (int64_t)sh.ncmb * b;
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  char *w = static_cast<char *>(ws);
  MbWs o;
  o.part = reinterpret_cast<float *>(w);
  w += al((size_t)sh.chunks * sh.rpad * ncol * sizeof(float));
  o.D = reinterpret_cast<float *>(w);
  w += al((size_t)ncol * sh.jp * sizeof(float));
  o.H = reinterpret_cast<__bf16 *>(w);
  w += al((size_t)ncol * sh.jp * sizeof(__bf16));
  o.Lo = reinterpret_cast<__bf16 *>(w);
  return o;
}

static bool mb_aligned16(const void *p, int64_t ld) {
  return ((reinterpret_cast<uintptr_t>(p) & 15) == 0) && (ld % 4 == 0);
}

template <int MODE, int NBW>
static void launch_mb_partial(bool vec, dim3 grid, dim3 block, hipStream_t st, const float *x, int64_t ldx, int N,
                              int b, const MbU &u, int r, const float *M, int64_t ldm, const MbShape &sh,
                              float *part) {
  const char *name = MODE == 0 ? "mb_partial" : "mb_partial_bf16x3";
  (void)ldm;
  if (vec)
    SLP_LAUNCH(name, (k_mb_partial<MODE, NBW, true>), grid, block, sh.lds_bytes, st, x, ldx, N, b, u.U32b, u.Uh,
               u.Ul, r, M, sh.ncmb, sh.logG, sh.nsg, sh.nw, sh.steps, sh.ss, part, sh.rpad);
  else
    SLP_LAUNCH(name, (k_mb_partial<MODE, NBW, false>), grid, block, sh.lds_bytes, st, x, ldx, N, b, u.U32b, u.Uh,
               u.Ul, r, M, sh.ncmb, sh.logG, sh.nsg, sh.nw, sh.steps, sh.ss, part, sh.rpad);
}

template <int MODE, int RK, int T, int CU>
static void launch_mb_apply(hipStream_t st, float *y, int64_t ldy, int N, int b, const MbU &u, const float *M,
                            int64_t ldm, int ncmb, const MbWs &w) {
  const dim3 grid((unsigned)((N + 64 * T - 1) / (64 * T)), (unsigned)((b + 15) / 16));
  (void)ldm;
  SLP_LAUNCH(MODE == 0 ? "mb_apply" : "mb_apply_bf16x3", (k_mb_apply<MODE, RK, T, CU>), grid, dim3(256), 0, st, y,
             ldy, N, b, u.T32, u.Th, u.Tl, M, ncmb, w.D, w.H, w.Lo);
}

template <int MODE>
static hipError_t launch_mb_apply_shape(const MbShape &sh, hipStream_t st, float *y, int64_t ldy, int N, int b,
                                        const MbU &u, const float *M, int64_t ldm, const MbWs &w) {
  const int rk = sh.jp / 32;
  if (rk == 1) {
    if (sh.tiles == 8 && sh.cu == 1) launch_mb_apply<MODE, 1, 8, 1>(st, y, ldy, N, b, u, M, ldm, sh.ncmb, w);
    else if (sh.tiles == 8) launch_mb_apply<MODE, 1, 8, 4>(st, y, ldy, N, b, u, M, ldm, sh.ncmb, w);
    else if (sh.cu == 1) launch_mb_apply<MODE, 1, 4, 1>(st, y, ldy, N, b, u, M, ldm, sh.ncmb, w);
    else launch_mb_apply<MODE, 1, 4, 4>(st, y, ldy, N, b, u, M, ldm, sh.ncmb, w);
  } else if (rk == 2) {
    launch_mb_apply<MODE, 2, 4, 1>(st, y, ldy, N, b, u, M, ldm, sh.ncmb, w);
  } else if (rk == 3) {
    launch_mb_apply<MODE, 3, 2, 1>(st, y, ldy, N, b, u, M, ldm, sh.ncmb, w);
  } else if (rk == 4) {
    launch_mb_apply<MODE, 4, 2, 1>(st, y, ldy, N, b, u, M, ldm, sh.ncmb, w);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mb_coeffs(int mode, const float *x, int64_t ldx, int64_t N, int64_t b, const MbU &u, int r,
                     const float *d, const float *M, int64_t ldm, const BandSet &bs, const MbShape &sh, const MbWs &w,
                     hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  if (!mb_ok(sh, N, b, r)) return hipErrorInvalidValue;
  const int64_t ncol = (int64_t)sh.ncmb * b;
  const dim3 gp((unsigned)sh.chunks, (unsigned)(sh.nsg * sh.ncg), (unsigned)sh.nz);
  const dim3 bp((unsigned)(64 * sh.nw));
  const bool vec = mb_aligned16(x, ldx);
  if (mode == 0) {
    if (sh.nbw == 2) launch_mb_partial<0, 2>(vec, gp, bp, st, x, ldx, (int)N, (int)b, u, r, M, ldm, sh, w.part);
    else launch_mb_partial<0, 1>(vec, gp, bp, st, x, ldx, (int)N, (int)b, u, r, M, ldm, sh, w.part);
  } else {
    if (sh.nbw == 2) launch_mb_partial<1, 2>(vec, gp, bp, st, x, ldx, (int)N, (int)b, u, r, M, ldm, sh, w.part);
    else launch_mb_partial<1, 1>(vec, gp, bp, st, x, ldx, (int)N, (int)b, u, r, M, ldm, sh, w.part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t outs = ncol * sh.jp;
  SLP_LAUNCH("mb_reduce", k_mb_reduce, dim3((unsigned)((outs + 15) / 16)), dim3(256), 0, st, w.part, sh.chunks,
             sh.rpad, (int)ncol, (int)b, r, sh.jp, d, w.D, w.H, w.Lo, bs);
  return hipGetLastError();
}

hipError_t mb_apply(int mode, float *y, int64_t ldy, int64_t N, int64_t b, const MbU &u, int r, const float *M,
                    int64_t ldm, const MbShape &sh, const MbWs &w, hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  if (!mb_ok(sh, N, b, r)) return hipErrorInvalidValue;
  if (mode == 0) return launch_mb_apply_shape<0>(sh, st, y, ldy, (int)N, (int)b, u, M, ldm, w);
  return launch_mb_apply_shape<1>(sh, st, y, ldy, (int)N, (int)b, u, M, ldm, w);
}

}  // namespace slp

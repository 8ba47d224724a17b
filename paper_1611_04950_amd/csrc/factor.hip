// Pieces of the fast factorization S_K S_K^T ~= T1 T2^T (Section 1.3, built
// on Theorem 1) that are not FFT passes: the Toeplitz kernel of B - F F^*
// for the setup, the random start block of its subspace iteration, a column
// sign convention, and the conversion between the FFT's packed pair bins and
// the real compressed coefficients.
//
// F is used in its real form F_r: columns 1/sqrt(N), then sqrt(2/N) cos(2 pi k n / N)
// and -sqrt(2/N) sin(2 pi k n / N) for k = 1 .. M, M = (kf - 1)/2, so that
// with X(k) = sum_n x[n] e^{-2 pi i k n / N}:
//   c[0] = X(0) / sqrt(N),  c[2k-1] = sqrt(2/N) Re X(k),  c[2k] = sqrt(2/N) Im X(k).
// The FFT passes transform the pair z = x1 + i x2 and keep Z(k) for |k| <= M
// at slot M + k of the pair's kf bins.
#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

// Circulant embedding (length L >= 2N) of the first column of B - F F^*:
// t(m) = sin(2 pi W m)/(pi m) - sin(pi kf m / N)/(N sin(pi m / N)), t(0) = 2W - kf/N.
__global__ void k_diff_embed(double *__restrict__ c, int64_t L, int64_t N, double W, int kf) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const int64_t kk = k > L - N ? L - k : k;
  double v = 0.0;
  if (kk == 0) {
    v = 2.0 * W - (double)kf / (double)N;
  } else if (kk < N) {
    const double m = (double)kk;
    v = sinpi(2.0 * W * m) / (M_PI * m) - sinpi((double)kf * m / (double)N) / ((double)N * sinpi(m / (double)N));
  }
  c[k] = v;
}

hipError_t diff_embed(double *c, int64_t L, int64_t N, double W, int kf, hipStream_t st) {
  hipLaunchKernelGGL(k_diff_embed, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, st, c, L, N, W, kf);
  return hipGetLastError();
}

// O[i + j ld] = +-1 from SplitMix64 (Steele, Lea and Flood, 2014) of the
// counter seed + j N + i: a reproducible random start block.
__global__ void k_rademacher(double *__restrict__ O, int64_t ld, int64_t N, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= N) return;
  uint64_t z = seed + (uint64_t)(j * N + i) * 0x9e3779b97f4a7c15ull + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  O[j * ld + i] = (z >> 63) ? 1.0 : -1.0;
}

hipError_t rademacher(double *O, int64_t ld, int64_t N, int64_t p, uint64_t seed, hipStream_t st) {
  if (N == 0 || p == 0) return hipSuccess;
  if (p > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rademacher, dim3((unsigned)((N + 255) / 256), (unsigned)p), dim3(256), 0, st, O, ld, N, seed);
  return hipGetLastError();
}

// Column j of V (N rows, leading dimension ld) negated unless its first entry
// of magnitude >= 1e-3 of the column's largest is positive.  One workgroup
// per column: a max reduction, then a min reduction of the first such index.
__global__ __launch_bounds__(256) void k_sign_fix(double *__restrict__ V, int64_t ld, int64_t N) {
  __shared__ double red[256];
  __shared__ int64_t ired[256];
  double *v = V + (int64_t)blockIdx.x * ld;
  const int t = threadIdx.x;
  double m = 0.0;
  for (int64_t i = t; i < N; i += 256) m = fmax(m, fabs(v[i]));
  red[t] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  const double thr = 1e-3 * red[0];
  int64_t first = N;
  for (int64_t i = t; i < N; i += 256)
    if (fabs(v[i]) >= thr) {
      first = i;
      break;
    }
  ired[t] = first;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) ired[t] = ired[t] < ired[t + s] ? ired[t] : ired[t + s];
    __syncthreads();
  }
  const int64_t f = ired[0];
  const bool flip = f < N && v[f] < 0.0 && red[0] > 0.0;
  __syncthreads();
  if (flip)
    for (int64_t i = t; i < N; i += 256) v[i] = -v[i];
}

hipError_t sign_fix_cols(double *V, int64_t ld, int64_t N, int64_t cols, hipStream_t st) {
  if (cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sign_fix, dim3((unsigned)cols), dim3(256), 0, st, V, ld, N);
  return hipGetLastError();
}

// R[:, j] -= mu[j] V[:, j] (N x r, leading dimension ld): the Ritz residuals
// T v_j - mu_j v_j once R holds T V.
__global__ void k_ritz_residual(double *__restrict__ R, const double *__restrict__ V, const double *__restrict__ mu,
                                int64_t ld, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= N) return;
  R[j * ld + i] -= mu[j] * V[j * ld + i];
}

hipError_t ritz_residual(double *R, const double *V, const double *mu, int64_t ld, int64_t N, int64_t r,
                         hipStream_t st) {
  if (N == 0 || r == 0) return hipSuccess;
  if (r > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ritz_residual, dim3((unsigned)((N + 255) / 256), (unsigned)r), dim3(256), 0, st, R, V, mu, ld,
                     N);
  return hipGetLastError();
}

// Pair bins -> real coefficients of both signals (rows 0 .. kf-1 of c):
// X1(k) = (Z(k) + conj Z(-k)) / 2, X2(k) = (Z(k) - conj Z(-k)) / 2i.
__global__ void k_bins_unpack(const cpx<float> *__restrict__ Zb, int kf, int64_t N, int b, int p0,
                              float *__restrict__ c, int64_t ldc) {
  const int M = (kf - 1) / 2;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = p0 + blockIdx.y;
  if (k > M) return;
  const cpx<float> A = Zb[(int64_t)p * kf + M + k], B = Zb[(int64_t)p * kf + M - k];
  const int s0 = 2 * p, s1 = 2 * p + 1;
  float *c0 = c + (int64_t)s0 * ldc, *c1 = c + (int64_t)s1 * ldc;
  if (k == 0) {
    const float sc = (float)(1.0 / sqrt((double)N));
    c0[0] = A.x * sc;
    if (s1 < b) c1[0] = A.y * sc;
    return;
  }
  const float sc = (float)sqrt(2.0 / (double)N) * 0.5f;
  c0[2 * k - 1] = (A.x + B.x) * sc;
  c0[2 * k] = (A.y - B.y) * sc;
  if (s1 < b) {
    c1[2 * k - 1] = (A.y + B.y) * sc;
    c1[2 * k] = (B.x - A.x) * sc;
  }
}

hipError_t bins_unpack(const cpx<float> *Zb, int kf, int64_t N, int64_t b, float *c, int64_t ldc, hipStream_t st) {
  const int64_t pairs = (b + 1) / 2;
  const int M = (kf - 1) / 2;
  for (int64_t p0 = 0; p0 < pairs; p0 += 65535) {
    const int64_t np = pairs - p0 < 65535 ? pairs - p0 : 65535;
    SLP_LAUNCH("bins_unpack", k_bins_unpack, dim3((unsigned)((M + 256) / 256), (unsigned)np), dim3(256), 0, st, Zb,
               kf, N, (int)b, (int)p0, c, ldc);
  }
  return hipGetLastError();
}

// Recovery's two reads of c in one launch.  Workgroups [0, nbp) (per_pair
// workgroups of 256 bins per pair) turn the real coefficients of both
// signals into pair bins scaled for an unnormalised inverse transform of
// length 2N: with Y(0) = sqrt(N) c[0] and Y(k) = sqrt(N/2) (c[2k-1] + i c[2k]),
// Z(k) = (Y1(k) + i Y2(k)) / N and Z(-k) = (conj Y1(k) + i conj Y2(k)) / N.
// The rest form dC[j b + s] = w[j] c[kf + j + s ldc] for j < r, s < b.
__global__ __launch_bounds__(256) void k_pack_scale(const float *__restrict__ c, int64_t ldc, int kf, int64_t N,
                                                    int b, int per_pair, int64_t nbp, cpx<float> *__restrict__ Zb,
                                                    int r, const float *__restrict__ w, float *__restrict__ dC) {
  const int64_t bid = blockIdx.x;
  if (bid < nbp) {
    const int M = (kf - 1) / 2;
    const int p = (int)(bid / per_pair);
    const int k = (int)(bid % per_pair) * 256 + threadIdx.x;
    if (k > M) return;
    const int s0 = 2 * p, s1 = 2 * p + 1;
    const bool has1 = s1 < b;
    const float *c0 = c + (int64_t)s0 * ldc, *c1 = c + (int64_t)(has1 ? s1 : s0) * ldc;
    cpx<float> *z = Zb + (int64_t)p * kf;
    if (k == 0) {
      const float sc = (float)(1.0 / sqrt((double)N));
      z[M] = cpx<float>{c0[0] * sc, has1 ? c1[0] * sc : 0.f};
      return;
    }
    const float f = (float)(1.0 / sqrt(2.0 * (double)N));
    const float a1 = c0[2 * k - 1], b1 = c0[2 * k];
    const float a2 = has1 ? c1[2 * k - 1] : 0.f, b2 = has1 ? c1[2 * k] : 0.f;
    z[M + k] = cpx<float>{(a1 - b2) * f, (b1 + a2) * f};
    z[M - k] = cpx<float>{(a1 + b2) * f, (a2 - b1) * f};
    return;
  }
  const int64_t o = (bid - nbp) * 256 + threadIdx.x;
  if (o >= (int64_t)r * b) return;
  const int64_t j = o / b, s = o % b;
  dC[o] = w[j] * c[kf + j + s * ldc];
}

hipError_t pack_scale(const float *c, int64_t ldc, int kf, int64_t N, int64_t b, cpx<float> *Zb, int r,
                      const float *w, float *dC, hipStream_t st) {
  const int64_t pairs = (b + 1) / 2;
  if (pairs == 0) return hipSuccess;
  const int M = (kf - 1) / 2;
  const int per_pair = (M + 256) / 256;
  const int64_t nbp = (int64_t)per_pair * pairs;
  const int64_t nbs = ((int64_t)r * b + 255) / 256;
  if (nbp + nbs > 0x7fffffffLL) return hipErrorInvalidValue;
  SLP_LAUNCH("pack_scale", k_pack_scale, dim3((unsigned)(nbp + nbs)), dim3(256), 0, st, c, ldc, kf, N, (int)b,
             per_pair, nbp, Zb, r, w, dC);
  return hipGetLastError();
}

}  // namespace slp

namespace slp {

// Theorem 1's factor of B - F F^* (Section 2, "Putting it all together"),
// in the real form used for real signals.  The construction's complex
// columns come in conjugate pairs, so row n of the real factors holds, for
// the first member of each pair, Re and Im of the compression column (L2)
// and twice Re and Im of the recovery column (L1):
//   group 1: L2 = D_A J Z,         L1 = D_A Z / (2 pi j)      (rH columns)
//   group 2: L2 = D_A Z,           L1 = -D_A J Z / (2 pi j)   (rH columns)
//   group 5: L2 = D_A V_A C_A^T,   L1 = D_A V_A / (2 j)       (2 rA columns)
//   group 7: L2 = D_B V_B C_B^T,   L1 = D_B V_B / 2           (2 rB - 1 columns)
// with D_A = e^{j pi kf n / N} (2 pi W' n, 2NW' = kf), D_B = e^{j pi (W + W') n},
// Z the CF-ADI factor of the Hilbert matrix (A = diag(n + 1/2), shifts p_k):
//   Z_1 = sqrt(2 p_1) / (n + 1/2 + p_1),
//   Z_k = sqrt(p_k / p_{k-1}) (n + 1/2 - p_{k-1}) / (n + 1/2 + p_k) Z_{k-1},
// (J Z)[n] = Z[N - 1 - n], and V_A, V_B the monomials u^i of the centred index
// u = (n - (N-1)/2) / N.  Columns: [Re of groups 1, 2, 5, 7 | Im of the same].
// FP64 arithmetic, FP32 results; one thread per n.
__global__ void k_theorem1_rows(int64_t N, int kf, double W, int rH, int rA, int rB,
                                const double *__restrict__ prm, float *__restrict__ L2, float *__restrict__ L1,
                                int64_t ld) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double *p = prm;
  const double *CA = prm + rH;
  const int na = 2 * rA, nb = 2 * rB - 1;
  const double *CB = CA + (int64_t)na * na;
  const int half = 2 * rH + na + nb;
  // D_A: angle pi (kf n mod 2N) / N;  D_B: angle pi ((W n mod 2) + (kf n mod 4N) / (2N))
  const int64_t kn = (int64_t)kf * n;
  double sa, ca, sb, cb;
  sincospi((double)(kn % (2 * N)) / (double)N, &sa, &ca);
  double tb = fmod(W * (double)n, 2.0) + (double)(kn % (4 * N)) / (double)(2 * N);
  sincospi(fmod(tb, 2.0), &sb, &cb);
  float *l2r = L2 + n, *l2i = L2 + n + (int64_t)half * ld;
  float *l1r = L1 + n, *l1i = L1 + n + (int64_t)half * ld;
  // Hilbert factor at n and at N - 1 - n
  const double al = (double)n + 0.5, alj = (double)(N - 1 - n) + 0.5;
  double z = 0.0, zj = 0.0;
  for (int k = 0; k < rH; ++k) {
    if (k == 0) {
      const double s0 = sqrt(2.0 * p[0]);
      z = s0 / (al + p[0]);
      zj = s0 / (alj + p[0]);
    } else {
      const double f = sqrt(p[k] / p[k - 1]);
      z *= f * (al - p[k - 1]) / (al + p[k]);
      zj *= f * (alj - p[k - 1]) / (alj + p[k]);
    }
    const int64_t c1 = (int64_t)k * ld, c2 = (int64_t)(rH + k) * ld;
    l2r[c1] = (float)(zj * ca);
    l2i[c1] = (float)(zj * sa);
    l1r[c1] = (float)(z * sa * M_1_PI);
    l1i[c1] = (float)(-z * ca * M_1_PI);
    l2r[c2] = (float)(z * ca);
    l2i[c2] = (float)(z * sa);
    l1r[c2] = (float)(-zj * sa * M_1_PI);
    l1i[c2] = (float)(zj * ca * M_1_PI);
  }
  // polynomial factors of A1 and B0
  const double u = ((double)n - 0.5 * (double)(N - 1)) / (double)N;
  double ui = 1.0;
  for (int i = 0; i < na; ++i) {
    double w = 0.0;  // (V_A C_A^T)[n, i] = sum_l C_A[i, l] u^l (Horner)
    for (int l = na - 1; l >= 0; --l) w = w * u + CA[(int64_t)i * na + l];
    const int64_t c = (int64_t)(2 * rH + i) * ld;
    l2r[c] = (float)(w * ca);
    l2i[c] = (float)(w * sa);
    l1r[c] = (float)(ui * sa);
    l1i[c] = (float)(-ui * ca);
    ui *= u;
  }
  ui = 1.0;
  for (int i = 0; i < nb; ++i) {
    double w = 0.0;
    for (int l = nb - 1; l >= 0; --l) w = w * u + CB[(int64_t)i * nb + l];
    const int64_t c = (int64_t)(2 * rH + na + i) * ld;
    l2r[c] = (float)(w * cb);
    l2i[c] = (float)(w * sb);
    l1r[c] = (float)(ui * cb);
    l1i[c] = (float)(ui * sb);
    ui *= u;
  }
}

hipError_t theorem1_rows(int64_t N, int kf, double W, int rH, int rA, int rB, const double *prm, float *L2,
                         float *L1, int64_t ld, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_theorem1_rows, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, kf, W, rH, rA, rB, prm,
                     L2, L1, ld);
  return hipGetLastError();
}

}  // namespace slp

// FP64 setup kernels: the Slepian vectors of the transition region.
//
// The paper precomputes the Slepian vectors whose eigenvalues lie in
// (eps, 1 - eps) (Section 2.3, "fast precomputation"; Section 4.1) and cites
// Slepian 1978 for the DPSS.  There, the DPSS are also the eigenvectors of a
// symmetric tridiagonal matrix T that commutes with B:
//     T[n,n]   = ((N-1)/2 - n)^2 cos(2 pi W),   n = 0..N-1
//     T[n,n+1] = (n+1)(N-1-n)/2,                 n = 0..N-2
// whose eigenvalues are well separated (B's are not), ordered so that the
// largest eigenvalue of T belongs to l = 0.  The GPU finds the eigenvalues of
// T for a window of indices around K by multisection on Sturm counts (one
// workgroup per eigenvalue, 256 trial points per round), the vectors by
// inverse iteration (one lane per vector, Gaussian elimination with partial
// pivoting of T - theta I), and B's eigenvalues as Rayleigh quotients
// lambda = s^T B s with B applied in FP64 by the FFT product.
#include <cfloat>
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace slp {

__global__ void k_tridiag_build(double *__restrict__ a, double *__restrict__ e2, int64_t N, double cw) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double h = 0.5 * (double)(N - 1) - (double)n;
  a[n] = h * h * cw;
  if (n < N - 1) {
    const double o = 0.5 * (double)(n + 1) * (double)(N - 1 - n);
    e2[n] = o * o;
  }
}

hipError_t tridiag_build(double *a, double *e2, int64_t N, double W, hipStream_t st) {
  const double cs = std::cos(2.0 * M_PI * W);
  hipLaunchKernelGGL(k_tridiag_build, dim3((N + 255) / 256), dim3(256), 0, st, a, e2, N, cs);
  return hipGetLastError();
}

// Number of eigenvalues of T below x: the count of negative pivots of the
// LDL^T factorisation of T - x I (Sturm sequence).
__device__ __forceinline__ int sturm_count(const double *__restrict__ a, const double *__restrict__ e2,
                                           int64_t N, double x, double pivmin) {
  double q = a[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int64_t k = 1; k < N; ++k) {
    q = (a[k] - x) - e2[k - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// One workgroup per eigenvalue theta_t (ascending index t): keep
// [lo, hi) with count(lo) <= t < count(hi) and split it at blockDim.x points
// per round until it is as narrow as FP64 allows.
__global__ __launch_bounds__(256) void k_bisect(const double *__restrict__ a, const double *__restrict__ e2,
                                                int64_t N, double gl, double gu, double pivmin, double atol,
                                                int64_t t0, double *__restrict__ theta) {
  __shared__ int first;
  const int64_t t = t0 + blockIdx.x;
  const int P = blockDim.x;
  double lo = gl, hi = gu;
  for (int round = 0; round < 24; ++round) {
    const double w = hi - lo;
    if (w <= atol + 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi))) break;
    const double xi = lo + w * (double)(threadIdx.x + 1) / (double)(P + 1);
    const int c = (xi < hi && xi > lo) ? sturm_count(a, e2, N, xi, pivmin) : (xi >= hi ? (int)N : 0);
    if (threadIdx.x == 0) first = P;
    __syncthreads();
    if ((int64_t)c > t) atomicMin(&first, (int)threadIdx.x);
    __syncthreads();
    const int f = first;
    const double nlo = f == 0 ? lo : lo + w * (double)f / (double)(P + 1);
    const double nhi = f == P ? hi : lo + w * (double)(f + 1) / (double)(P + 1);
    lo = nlo;
    hi = nhi;
    __syncthreads();
  }
  if (threadIdx.x == 0) theta[blockIdx.x] = 0.5 * (lo + hi);
}

hipError_t tridiag_bisect(const double *a, const double *e2, int64_t N, double gl, double gu, double pivmin,
                          int64_t t0, int64_t count, double *theta, hipStream_t st) {
  const double atol = DBL_EPSILON * fmax(fabs(gl), fabs(gu));
  hipLaunchKernelGGL(k_bisect, dim3((unsigned)count), dim3(256), 0, st, a, e2, N, gl, gu, pivmin, atol, t0,
                     theta);
  return hipGetLastError();
}

// Scratch of inverse iteration, interleaved [k][vector] so that the lanes of
// a wavefront (one vector each) touch consecutive addresses.
struct InvScratch {
  double *dl, *d, *du, *du2, *x;
  unsigned char *piv;
};

static InvScratch carve(void *p, int64_t N, int64_t count) {
  InvScratch s;
  const size_t nd = (size_t)N * (size_t)count;
  double *q = (double *)p;
  s.dl = q;
  s.d = q + nd;
  s.du = q + 2 * nd;
  s.du2 = q + 3 * nd;
  s.x = q + 4 * nd;
  s.piv = (unsigned char *)(q + 5 * nd);
  return s;
}

size_t inviter_scratch_bytes(int64_t N, int64_t count) {
  return (size_t)N * (size_t)count * (5 * sizeof(double) + 1) + 256;
}

__device__ __forceinline__ double start_value(int64_t k, int64_t j) {
  uint32_t h = (uint32_t)(k * 2654435761ull) ^ (uint32_t)(j * 40503u + 0x9e3779b9u);
  h ^= h >> 16;
  h *= 0x7feb352du;
  h ^= h >> 15;
  return 0.5 + (double)(h & 0xffffu) / 65536.0;
}

// One lane per eigenvalue: factor T - theta I = P L U (partial pivoting,
// U with two superdiagonals), then `iters` rounds of x <- (T - theta I)^{-1} x
// with normalisation.  The final (unnormalised) iterate is left in s.x.
__global__ __launch_bounds__(64) void k_inviter(const double *__restrict__ a, const double *__restrict__ off,
                                                int64_t N, const double *__restrict__ theta, int64_t count,
                                                InvScratch s, double tiny, int iters) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  const double th = theta[j];
  const int64_t C = count;
  double cur_d = a[0] - th;
  double cur_du = N > 1 ? off[0] : 0.0;
  for (int64_t k = 0; k < N - 1; ++k) {
    const double sub = off[k];
    const double nd = a[k + 1] - th;
    const double nu = k < N - 2 ? off[k + 1] : 0.0;
    const int64_t o = k * C + j;
    if (fabs(cur_d) >= fabs(sub)) {
      double dk = cur_d;
      if (dk == 0.0) dk = tiny;
      const double f = sub / dk;
      s.d[o] = dk;
      s.du[o] = cur_du;
      s.du2[o] = 0.0;
      s.dl[o] = f;
      s.piv[o] = 0;
      cur_d = nd - f * cur_du;
      cur_du = nu;
    } else {
      const double f = cur_d / sub;
      s.d[o] = sub;
      s.du[o] = nd;
      s.du2[o] = nu;
      s.dl[o] = f;
      s.piv[o] = 1;
      cur_d = cur_du - f * nd;
      cur_du = -f * nu;
    }
  }
  if (cur_d == 0.0) cur_d = tiny;
  s.d[(N - 1) * C + j] = cur_d;
  for (int64_t k = 0; k < N; ++k) s.x[k * C + j] = start_value(k, j);
  double scale = 1.0;
  for (int it = 0; it < iters; ++it) {
    // forward: apply P and L^{-1}
    double prev = s.x[j] * scale;
    for (int64_t k = 0; k < N - 1; ++k) {
      const int64_t o = k * C + j;
      double nxt = s.x[o + C] * scale;
      const double f = s.dl[o];
      if (s.piv[o] == 0) {
        s.x[o] = prev;
        nxt -= f * prev;
      } else {
        s.x[o] = nxt;
        nxt = prev - f * nxt;
      }
      prev = nxt;
    }
    s.x[(N - 1) * C + j] = prev;
    // back substitution with U
    double x2 = 0.0, x1 = 0.0, ss = 0.0;
    for (int64_t k = N - 1; k >= 0; --k) {
      const int64_t o = k * C + j;
      double v = s.x[o];
      if (k < N - 1) v -= s.du[o] * x1;
      if (k < N - 2) v -= s.du2[o] * x2;
      v /= s.d[o];
      s.x[o] = v;
      ss += v * v;
      x2 = x1;
      x1 = v;
    }
    scale = 1.0 / sqrt(ss);
  }
}

// Normalise to unit 2-norm, sign so that the first entry of magnitude
// >= 1e-3 max|v| is positive, and write column count-1-j of V.
__global__ __launch_bounds__(256) void k_normalize(InvScratch s, int64_t N, int64_t count, double *__restrict__ V) {
  __shared__ double red[256];
  __shared__ int64_t redi[256];
  const int64_t j = blockIdx.x;
  const int64_t C = count;
  double ss = 0.0, mx = 0.0;
  for (int64_t k = threadIdx.x; k < N; k += blockDim.x) {
    const double v = s.x[k * C + j];
    ss += v * v;
    mx = fmax(mx, fabs(v));
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double tot = red[0];
  __syncthreads();
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double vmax = red[0];
  int64_t first = N;
  for (int64_t k = threadIdx.x; k < N; k += blockDim.x) {
    if (fabs(s.x[k * C + j]) >= 1e-3 * vmax) {
      first = k;
      break;
    }
  }
  redi[threadIdx.x] = first;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) redi[threadIdx.x] = redi[threadIdx.x] < redi[threadIdx.x + w] ? redi[threadIdx.x] : redi[threadIdx.x + w];
    __syncthreads();
  }
  const int64_t f = redi[0];
  const double sg = (f < N && s.x[f * C + j] < 0.0) ? -1.0 : 1.0;
  const double sc = sg / sqrt(tot);
  double *out = V + (count - 1 - j) * N;
  for (int64_t k = threadIdx.x; k < N; k += blockDim.x) out[k] = s.x[k * C + j] * sc;
}

hipError_t tridiag_inviter(const double *a, const double *off, int64_t N, const double *theta, int64_t count,
                           double *V, void *scratch, int iters, hipStream_t st) {
  InvScratch s = carve(scratch, N, count);
  // a zero pivot is replaced by eps * ||T|| (T's entries are at most N^2/4)
  const double tiny = DBL_EPSILON * 0.25 * (double)N * (double)N;
  hipLaunchKernelGGL(k_inviter, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, st, a, off, N, theta, count, s,
                     tiny, iters);
  hipLaunchKernelGGL(k_normalize, dim3((unsigned)count), dim3(256), 0, st, s, N, count, V);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_rayleigh(const double *__restrict__ V, const double *__restrict__ BV,
                                                  int64_t N, double *__restrict__ lam, double *__restrict__ res) {
  __shared__ double red[256];
  const int64_t j = blockIdx.x;
  const double *v = V + j * N;
  const double *bv = BV + j * N;
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < N; k += blockDim.x) acc += v[k] * bv[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double l = red[0];
  __syncthreads();
  acc = 0.0;
  for (int64_t k = threadIdx.x; k < N; k += blockDim.x) {
    const double r = bv[k] - l * v[k];
    acc += r * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lam[j] = l;
    res[j] = sqrt(red[0]);
  }
}

hipError_t rayleigh(const double *V, const double *BV, int64_t N, int64_t count, double *lam, double *res,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_rayleigh, dim3((unsigned)count), dim3(256), 0, st, V, BV, N, lam, res);
  return hipGetLastError();
}

template <typename A, typename B>
__global__ void k_cast(const A *__restrict__ src, int64_t lds, B *__restrict__ dst, int64_t ldd, int64_t rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i < rows) dst[c * ldd + i] = (B)src[c * lds + i];
}

hipError_t cast_f64_to_f32(const double *src, int64_t ld_src, float *dst, int64_t ld_dst, int64_t rows,
                           int64_t cols, hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast<double, float>), dim3((unsigned)((rows + 255) / 256), (unsigned)cols), dim3(256), 0,
                     st, src, ld_src, dst, ld_dst, rows);
  return hipGetLastError();
}

hipError_t cast_f32_to_f64(const float *src, int64_t ld_src, double *dst, int64_t ld_dst, int64_t rows,
                           int64_t cols, hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast<float, double>), dim3((unsigned)((rows + 255) / 256), (unsigned)cols), dim3(256), 0,
                     st, src, ld_src, dst, ld_dst, rows);
  return hipGetLastError();
}

}  // namespace slp

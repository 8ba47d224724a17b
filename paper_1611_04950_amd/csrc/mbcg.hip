// Conjugate gradients on the band-sum operator of a multiband dictionary
// (Section 1.4, application i): per signal s, with A the sum of the bands'
// fast projections (applied by the band-set kernels), solve A z = A x from
// z = 0, so that z is the orthogonal projection of x onto the span of the
// modulated Slepian bases.  The vector kernels below carry the per-signal
// scalars of the iteration in FP64 (dot products accumulated in FP64 over
// FP32 vectors, in a fixed order); every decision (step size, direction
// update, stopping) is taken on the device, one state record per signal:
//   a = rr / (p . Ap),  z += a p,  r -= a Ap,  beta = rr_new / rr,
//   p = r + beta p,  active while rr > tol^2 ||A x||^2.
#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

namespace {

constexpr int kDotThreads = 256;

// Sum of u[n] v[n] over chunk c (kCgChunk samples) of signal s, in FP64.
__global__ void __launch_bounds__(kDotThreads) k_cg_dot(const float *__restrict__ u, int64_t ldu,
                                                        const float *__restrict__ v, int64_t ldv, int64_t N,
                                                        double *__restrict__ part, int nch) {
  const int c = blockIdx.x, s = blockIdx.y;
  const int64_t n0 = (int64_t)c * kCgChunk;
  const int64_t n1 = n0 + kCgChunk < N ? n0 + kCgChunk : N;
  const float *us = u + (int64_t)s * ldu, *vs = v + (int64_t)s * ldv;
  double acc = 0.0;
  for (int64_t n = n0 + threadIdx.x; n < n1; n += kDotThreads) acc += (double)us[n] * (double)vs[n];
  __shared__ double red[kDotThreads];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)s * nch + c] = red[0];
}

__device__ __forceinline__ double chunk_sum(const double *__restrict__ part, int nch, int s) {
  double t = 0.0;
  for (int c = 0; c < nch; ++c) t += part[(int64_t)s * nch + c];
  return t;
}

// rr = ||r||^2 = ||A x||^2, active = rr > tol^2 rr (and rr > 0).
__global__ void k_cg_init(const double *__restrict__ part, int nch, int b, double tol, CgState *__restrict__ st) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b) return;
  const double rr = chunk_sum(part, nch, s);
  CgState q;
  q.rr = rr;
  q.nb2 = rr;
  q.a = 0.0;
  q.beta = 0.0;
  q.iters = 0;
  q.active = (rr > 0.0 && rr > tol * tol * rr) ? 1 : 0;
  q.upd = 0;
  st[s] = q;
}

// a = rr / (p . Ap) for the active signals (a breakdown, p . Ap <= 0, stops the signal).
__global__ void k_cg_alpha(const double *__restrict__ part, int nch, int b, CgState *__restrict__ st) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b) return;
  CgState q = st[s];
  const double pap = chunk_sum(part, nch, s);
  if (q.active && pap > 0.0) {
    q.a = q.rr / pap;
  } else {
    q.a = 0.0;
    q.active = 0;
  }
  st[s] = q;
}

// z += a p; r -= a Ap; chunk partials of ||r||^2.
__global__ void __launch_bounds__(kDotThreads) k_cg_update(float *__restrict__ z, int64_t ldz,
                                                           float *__restrict__ r, const float *__restrict__ p,
                                                           const float *__restrict__ ap, int64_t ldw, int64_t N,
                                                           const CgState *__restrict__ st, double *__restrict__ part,
                                                           int nch) {
  const int c = blockIdx.x, s = blockIdx.y;
  const double a = st[s].a;
  const int64_t n0 = (int64_t)c * kCgChunk;
  const int64_t n1 = n0 + kCgChunk < N ? n0 + kCgChunk : N;
  float *zs = z + (int64_t)s * ldz;
  float *rs = r + (int64_t)s * ldw;
  const float *ps = p + (int64_t)s * ldw, *as = ap + (int64_t)s * ldw;
  const float af = (float)a;
  double acc = 0.0;
  for (int64_t n = n0 + threadIdx.x; n < n1; n += kDotThreads) {
    float rv = rs[n];
    if (a != 0.0) {
      zs[n] = zs[n] + af * ps[n];
      rv = rv - af * as[n];
      rs[n] = rv;
    }
    acc += (double)rv * (double)rv;
  }
  __shared__ double red[kDotThreads];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)s * nch + c] = red[0];
}

// beta = rr_new / rr; the direction is updated for the signals that were
// active in this step; rr, the step count and the stopping test follow.
__global__ void k_cg_beta(const double *__restrict__ part, int nch, int b, double tol, CgState *__restrict__ st) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b) return;
  CgState q = st[s];
  q.upd = q.active;
  if (q.active) {
    const double rn = chunk_sum(part, nch, s);
    q.beta = rn / q.rr;
    q.rr = rn;
    q.iters += 1;
    q.active = q.rr > tol * tol * q.nb2 ? 1 : 0;
  } else {
    q.beta = 0.0;
  }
  st[s] = q;
}

// p = r + beta p for the signals updated in this step.
__global__ void __launch_bounds__(kDotThreads) k_cg_direction(float *__restrict__ p, const float *__restrict__ r,
                                                              int64_t ldw, int64_t N, const CgState *__restrict__ st) {
  const int s = blockIdx.y;
  if (!st[s].upd) return;
  const float bf = (float)st[s].beta;
  const int64_t n = (int64_t)blockIdx.x * kDotThreads + threadIdx.x;
  if (n >= N) return;
  p[(int64_t)s * ldw + n] = r[(int64_t)s * ldw + n] + bf * p[(int64_t)s * ldw + n];
}

__global__ void k_fill_zero(float *__restrict__ y, int64_t ldy, int64_t N) {
  const int64_t n = (int64_t)blockIdx.x * kDotThreads + threadIdx.x;
  if (n < N) y[(int64_t)blockIdx.y * ldy + n] = 0.0f;
}

__global__ void k_copy_rows(const float *__restrict__ src, int64_t lds, float *__restrict__ dst, int64_t ldd,
                            int64_t N) {
  const int64_t n = (int64_t)blockIdx.x * kDotThreads + threadIdx.x;
  if (n < N) dst[(int64_t)blockIdx.y * ldd + n] = src[(int64_t)blockIdx.y * lds + n];
}

}  // namespace

int cg_nchunks(int64_t N) { return (int)((N + kCgChunk - 1) / kCgChunk); }

hipError_t cg_dot(const float *u, int64_t ldu, const float *v, int64_t ldv, int64_t N, int64_t b, double *part,
                  hipStream_t st) {
  const int nch = cg_nchunks(N);
  SLP_LAUNCH("cg_dot", k_cg_dot, dim3((unsigned)nch, (unsigned)b), dim3(kDotThreads), 0, st, u, ldu, v, ldv, N,
             part, nch);
  return hipGetLastError();
}

hipError_t cg_init(const double *part, int64_t N, int64_t b, double tol, CgState *state, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_init, dim3((unsigned)((b + 63) / 64)), dim3(64), 0, st, part, cg_nchunks(N), (int)b, tol,
                     state);
  return hipGetLastError();
}

hipError_t cg_alpha(const double *part, int64_t N, int64_t b, CgState *state, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_alpha, dim3((unsigned)((b + 63) / 64)), dim3(64), 0, st, part, cg_nchunks(N), (int)b,
                     state);
  return hipGetLastError();
}

hipError_t cg_update(float *z, int64_t ldz, float *r, const float *p, const float *ap, int64_t ldw, int64_t N,
                     int64_t b, const CgState *state, double *part, hipStream_t st) {
  const int nch = cg_nchunks(N);
  SLP_LAUNCH("cg_update", k_cg_update, dim3((unsigned)nch, (unsigned)b), dim3(kDotThreads), 0, st, z, ldz, r, p, ap,
             ldw, N, state, part, nch);
  return hipGetLastError();
}

hipError_t cg_beta(const double *part, int64_t N, int64_t b, double tol, CgState *state, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_beta, dim3((unsigned)((b + 63) / 64)), dim3(64), 0, st, part, cg_nchunks(N), (int)b, tol,
                     state);
  return hipGetLastError();
}

hipError_t cg_direction(float *p, const float *r, int64_t ldw, int64_t N, int64_t b, const CgState *state,
                        hipStream_t st) {
  SLP_LAUNCH("cg_direction", k_cg_direction, dim3((unsigned)((N + kDotThreads - 1) / kDotThreads), (unsigned)b),
             dim3(kDotThreads), 0, st, p, r, ldw, N, state);
  return hipGetLastError();
}

hipError_t fill_zero_rows(float *y, int64_t ldy, int64_t N, int64_t b, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((N + kDotThreads - 1) / kDotThreads), (unsigned)b),
                     dim3(kDotThreads), 0, st, y, ldy, N);
  return hipGetLastError();
}

hipError_t copy_rows(const float *src, int64_t lds, float *dst, int64_t ldd, int64_t N, int64_t b, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((N + kDotThreads - 1) / kDotThreads), (unsigned)b),
                     dim3(kDotThreads), 0, st, src, lds, dst, ldd, N);
  return hipGetLastError();
}

}  // namespace slp

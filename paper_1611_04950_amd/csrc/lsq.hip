// Elementwise and reduction helpers of the least-squares refinement
// (Section 2.3 "Fast Tikhonov regularization"): the FP64 residual of the
// regularised normal equations (B^2 + alpha I) x = B y and its norms.
#include "common.h"
#include "kernels.h"

namespace slp {

__global__ void k_lsq_residual(const double *__restrict__ By, const double *__restrict__ u,
                               const double *__restrict__ x, int64_t ldx, double alpha,
                               double *__restrict__ rho, int64_t N) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = blockIdx.y;
  if (n >= N) return;
  const int64_t o = s * N + n;
  rho[o] = (By[o] - u[o]) - alpha * x[s * ldx + n];
}

hipError_t lsq_residual(const double *By, const double *u, const double *x, int64_t ldx, double alpha, double *rho,
                        int64_t N, int64_t b, hipStream_t st) {
  if (b == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lsq_residual, dim3((unsigned)((N + 255) / 256), (unsigned)b), dim3(256), 0, st, By, u, x,
                     ldx, alpha, rho, N);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_col_norms(const double *__restrict__ v, int64_t ldv, int64_t N,
                                                   double *__restrict__ norms) {
  __shared__ double red[256];
  const double *c = v + (int64_t)blockIdx.x * ldv;
  double acc = 0.0;
  for (int64_t n = threadIdx.x; n < N; n += 256) acc += c[n] * c[n];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[blockIdx.x] = sqrt(red[0]);
}

hipError_t col_norms(const double *v, int64_t ldv, int64_t N, int64_t b, double *norms, hipStream_t st) {
  if (b == 0) return hipSuccess;
  hipLaunchKernelGGL(k_col_norms, dim3((unsigned)b), dim3(256), 0, st, v, ldv, N, norms);
  return hipGetLastError();
}

__global__ void k_add_f32_to_f64(const float *__restrict__ e, int64_t lde, double *__restrict__ x, int64_t ldx,
                                 int64_t N) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = blockIdx.y;
  if (n < N) x[s * ldx + n] += (double)e[s * lde + n];
}

hipError_t add_f32_to_f64(const float *e, int64_t lde, double *x, int64_t ldx, int64_t N, int64_t b, hipStream_t st) {
  if (b == 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_f32_to_f64, dim3((unsigned)((N + 255) / 256), (unsigned)b), dim3(256), 0, st, e, lde, x,
                     ldx, N);
  return hipGetLastError();
}

}  // namespace slp

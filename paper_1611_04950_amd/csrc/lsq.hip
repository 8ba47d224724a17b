// Elementwise and reduction helpers of the least-squares refinement
// (Section 1.3 "Fast Tikhonov regularization"): the FP64 residual of the
// regularised normal equations (B^2 + alpha I) x = B y and its norms.
#include "common.h"
#include "kernels.h"

namespace slp {

// Column norms in two passes with a fixed summation order: pass 1 gives each
// of `parts` workgroups per column one contiguous segment (four independent
// accumulators per thread, then a tree over the workgroup), pass 2 sums a
// column's segment partials in order and takes the square root.
__global__ __launch_bounds__(256) void k_col_norms_part(const double *__restrict__ v, int64_t ldv, int64_t N,
                                                        int64_t seg, int parts, double *__restrict__ part) {
  __shared__ double red[256];
  const int p = blockIdx.x, s = blockIdx.y;
  const double *c = v + (int64_t)s * ldv;
  const int64_t n0 = (int64_t)p * seg, n1 = n0 + seg < N ? n0 + seg : N;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t n = n0 + threadIdx.x;
  for (; n + 768 < n1; n += 1024) {
    const double x0 = c[n], x1 = c[n + 256], x2 = c[n + 512], x3 = c[n + 768];
    a0 += x0 * x0;
    a1 += x1 * x1;
    a2 += x2 * x2;
    a3 += x3 * x3;
  }
  for (; n < n1; n += 256) a0 += c[n] * c[n];
  red[threadIdx.x] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)s * parts + p] = red[0];
}

__global__ __launch_bounds__(256) void k_col_norms_sum(const double *__restrict__ part, int parts,
                                                       double *__restrict__ norms) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  red[threadIdx.x] = (int)threadIdx.x < parts ? part[(int64_t)s * parts + threadIdx.x] : 0.0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[s] = sqrt(red[0]);
}

// The residual rho = (B y - u) - alpha x in one pass with its column norms:
// rho is formed in FP64 and written as FP32 (the input of the FP32 solve of
// the next sweep), and its squares are summed exactly as k_col_norms_part
// sums a stored column (same segments, accumulators and tree), so the norms
// equal col_norms of the FP64 residual.
__global__ __launch_bounds__(256) void k_lsq_residual_part(const double *__restrict__ By, const double *__restrict__ u,
                                                           const double *__restrict__ x, int64_t ldx, double alpha,
                                                           float *__restrict__ rho32, int64_t N, int64_t seg,
                                                           int parts, double *__restrict__ part) {
  __shared__ double red[256];
  const int p = blockIdx.x, s = blockIdx.y;
  const int64_t o = (int64_t)s * N;
  const double *xs = x + (int64_t)s * ldx;
  const int64_t n0 = (int64_t)p * seg, n1 = n0 + seg < N ? n0 + seg : N;
  auto res = [&](int64_t n) {
    const double r = (By[o + n] - u[o + n]) - alpha * xs[n];
    rho32[o + n] = (float)r;
    return r;
  };
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t n = n0 + threadIdx.x;
  for (; n + 768 < n1; n += 1024) {
    const double x0 = res(n), x1 = res(n + 256), x2 = res(n + 512), x3 = res(n + 768);
    a0 += x0 * x0;
    a1 += x1 * x1;
    a2 += x2 * x2;
    a3 += x3 * x3;
  }
  for (; n < n1; n += 256) {
    const double r = res(n);
    a0 += r * r;
  }
  red[threadIdx.x] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)s * parts + p] = red[0];
}

// Segments of col_norms: about 2048 workgroups over the batch, at most
// kNormParts per column, whole 1024-sample rounds.
static void norm_segments(int64_t N, int64_t b, int64_t &seg, int64_t &parts) {
  parts = 2048 / b;
  if (parts < 1) parts = 1;
  if (parts > kNormParts) parts = kNormParts;
  seg = (N + parts - 1) / parts;
  seg = (seg + 1023) / 1024 * 1024;
  parts = (N + seg - 1) / seg;
  if (parts < 1) parts = 1;
}

hipError_t lsq_residual_norms(const double *By, const double *u, const double *x, int64_t ldx, double alpha,
                              float *rho32, int64_t N, int64_t b, double *norms, double *part, hipStream_t st) {
  if (b == 0) return hipSuccess;
  if (b > 65535) {
    for (int64_t s0 = 0; s0 < b; s0 += 65535) {
      const int64_t bb = b - s0 < 65535 ? b - s0 : 65535;
      const hipError_t e = lsq_residual_norms(By + s0 * N, u + s0 * N, x + s0 * ldx, ldx, alpha, rho32 + s0 * N, N,
                                              bb, norms + s0, part + s0 * kNormParts, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  int64_t seg = 0, parts = 0;
  norm_segments(N, b, seg, parts);
  hipLaunchKernelGGL(k_lsq_residual_part, dim3((unsigned)parts, (unsigned)b), dim3(256), 0, st, By, u, x, ldx, alpha,
                     rho32, N, seg, (int)parts, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_norms_sum, dim3((unsigned)b), dim3(256), 0, st, part, (int)parts, norms);
  return hipGetLastError();
}

hipError_t col_norms(const double *v, int64_t ldv, int64_t N, int64_t b, double *norms, double *part,
                     hipStream_t st) {
  if (b == 0) return hipSuccess;
  if (b > 65535) {
    for (int64_t s0 = 0; s0 < b; s0 += 65535) {
      const int64_t bb = b - s0 < 65535 ? b - s0 : 65535;
      const hipError_t e = col_norms(v + s0 * ldv, ldv, N, bb, norms + s0, part + s0 * kNormParts, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  int64_t seg = 0, parts = 0;
  norm_segments(N, b, seg, parts);
  hipLaunchKernelGGL(k_col_norms_part, dim3((unsigned)parts, (unsigned)b), dim3(256), 0, st, v, ldv, N, seg,
                     (int)parts, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_norms_sum, dim3((unsigned)b), dim3(256), 0, st, part, (int)parts, norms);
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

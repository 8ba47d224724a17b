// The pseudoinverse's low-rank correction in FP64 (Corollary 3, Lemma 5):
//     x += U diag(d) U^T y,  d = 1/lambda - lambda on I2, -lambda on I3.
// The weights 1/lambda reach 1/eps at the edge of the transition set, so
// rounding in U^T y is amplified by up to that factor; the product runs in
// FP64 from the plan's FP64 vectors (the FFT product B y stays FP32, its
// rounding is not amplified).  C = U^T Y is split over chunks of samples,
// each workgroup forming 64 j x 32 signals of one chunk from LDS tiles, and
// the chunk partials are summed in a fixed order (deterministic).
#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

int corr_rpad(int r) { return (r + 31) / 32 * 32; }

constexpr int kC64Chunk = 1024;  // samples per workgroup
constexpr int kC64Sub = 64;      // samples staged in LDS at a time
constexpr int kC64Sig = 32;      // signals per workgroup

int corr64_chunks(int64_t N) { return (int)((N + kC64Chunk - 1) / kC64Chunk); }

// grid (chunks, ceil(b / 32)), 256 threads: thread t owns U column j0 + t % 64
// and signals 8 (t / 64) .. 8 (t / 64) + 7 of the workgroup's 32.
__global__ __launch_bounds__(256) void k_corr64_partial(const float *__restrict__ y, int64_t ldy, int N, int b,
                                                        const double *__restrict__ U, int64_t ldu, int r,
                                                        double *__restrict__ part) {
  __shared__ double Ut[64][kC64Sub + 1];
  __shared__ double Yt[kC64Sig][kC64Sub + 1];
  const int t = threadIdx.x, jj = t & 63, sp = t >> 6;
  const int s_base = blockIdx.y * kC64Sig;
  const int n_chunk = blockIdx.x * kC64Chunk;
  for (int j0 = 0; j0 < r; j0 += 64) {
    double a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = 0.0;
    for (int sub = 0; sub < kC64Chunk; sub += kC64Sub) {
      const int n0 = n_chunk + sub;
      if (n0 >= N) break;
      __syncthreads();
      for (int e = t; e < 64 * kC64Sub; e += 256) {
        const int j = e / kC64Sub, nn = e % kC64Sub, n = n0 + nn;
        Ut[j][nn] = (n < N && j0 + j < r) ? U[(int64_t)(j0 + j) * ldu + n] : 0.0;
      }
      for (int e = t; e < kC64Sig * kC64Sub; e += 256) {
        const int s = e / kC64Sub, nn = e % kC64Sub, n = n0 + nn;
        Yt[s][nn] = (n < N && s_base + s < b) ? (double)y[(int64_t)(s_base + s) * ldy + n] : 0.0;
      }
      __syncthreads();
#pragma unroll 4
      for (int nn = 0; nn < kC64Sub; ++nn) {
        const double u = Ut[jj][nn];
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] += u * Yt[8 * sp + q][nn];
      }
    }
    const int j = j0 + jj;
    if (j < r) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int s = s_base + 8 * sp + q;
        if (s < b) part[((int64_t)blockIdx.x * r + j) * b + s] = a[q];
      }
    }
  }
}

// dC[j][s] = d[j] * sum over chunks of part[chunk][j][s]: 16 outputs per
// workgroup, 16 lanes per output each summing every 16th chunk, then a
// fixed-order sum of the 16 through LDS.
__global__ __launch_bounds__(256) void k_corr64_reduce(const double *__restrict__ part, int chunks, int b, int r,
                                                       const double *__restrict__ d, double *__restrict__ dC) {
  __shared__ double red[16][17];
  const int og = threadIdx.x & 15, cg = threadIdx.x >> 4;
  const int64_t o = (int64_t)blockIdx.x * 16 + og;  // o = j b + s
  const bool valid = o < (int64_t)r * b;
  double acc = 0.0;
  if (valid) {
    const int64_t stride = (int64_t)r * b;
    for (int c = cg; c < chunks; c += 16) acc += part[(int64_t)c * stride + o];
  }
  red[cg][og] = acc;
  __syncthreads();
  if (cg == 0 && valid) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][og];
    dC[o] = d[o / b] * t;
  }
}

// x[s][n] += sum_j U[n][j] dC[j][s]: one sample per lane, 32 signals per
// workgroup, dC staged in LDS 64 columns at a time.
__global__ __launch_bounds__(256) void k_corr64_apply(double *__restrict__ x, int64_t ldx, int N, int b,
                                                      const double *__restrict__ U, int64_t ldu, int r,
                                                      const double *__restrict__ dC) {
  __shared__ double dcs[64][kC64Sig];
  const int n = blockIdx.x * 256 + threadIdx.x;
  const int s_base = blockIdx.y * kC64Sig;
  double acc[kC64Sig];
#pragma unroll
  for (int s = 0; s < kC64Sig; ++s) acc[s] = 0.0;
  for (int j0 = 0; j0 < r; j0 += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * kC64Sig; e += 256) {
      const int j = e / kC64Sig, s = e % kC64Sig;
      dcs[j][s] = (j0 + j < r && s_base + s < b) ? dC[(int64_t)(j0 + j) * b + s_base + s] : 0.0;
    }
    __syncthreads();
    if (n < N) {
      const int jn = r - j0 < 64 ? r - j0 : 64;
      for (int j = 0; j < jn; ++j) {
        const double u = U[(int64_t)(j0 + j) * ldu + n];
#pragma unroll
        for (int s = 0; s < kC64Sig; ++s) acc[s] += u * dcs[j][s];
      }
    }
  }
  if (n < N) {
#pragma unroll
    for (int s = 0; s < kC64Sig; ++s)
      if (s_base + s < b) x[(int64_t)(s_base + s) * ldx + n] += acc[s];
  }
}

hipError_t corr64(const float *y, int64_t ldy, double *x, int64_t ldx, int64_t N, int64_t b, const double *U,
                  int64_t ldu, int r, const double *d, double *part, double *dC, hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  if ((b + kC64Sig - 1) / kC64Sig > 65535) return hipErrorInvalidValue;
  const int chunks = corr64_chunks(N);
  const unsigned gy = (unsigned)((b + kC64Sig - 1) / kC64Sig);
  SLP_LAUNCH("corr64_partial", k_corr64_partial, dim3((unsigned)chunks, gy), dim3(256), 0, st, y, ldy, (int)N,
             (int)b, U, ldu, r, part);
  const int64_t outs = (int64_t)r * b;
  SLP_LAUNCH("corr64_reduce", k_corr64_reduce, dim3((unsigned)((outs + 15) / 16)), dim3(256), 0, st, part, chunks,
             (int)b, r, d, dC);
  SLP_LAUNCH("corr64_apply", k_corr64_apply, dim3((unsigned)((N + 255) / 256), gy), dim3(256), 0, st, x, ldx,
             (int)N, (int)b, U, ldu, r, dC);
  return hipGetLastError();
}

size_t corr64_workspace_doubles(int64_t N, int64_t b, int r) {
  return (size_t)corr64_chunks(N) * r * b + (size_t)r * b;
}

}  // namespace slp

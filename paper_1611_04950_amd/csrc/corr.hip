// Low-rank correction of the fast operators (Corollaries 2-4; Lemmas 5-7):
//     y += U diag(d) U^T x
// with U the N x r transition Slepian vectors.  C = U^T X is a tall-skinny
// product reduced over N (r x N by N x b); it is split over chunks of rows,
// each workgroup forming a 32 x 32 tile of C from LDS-staged slices of U and
// X, and the chunk partials are summed in a fixed order (deterministic).
#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

constexpr int kChunkRows = 1024;   // rows of N per workgroup in corr_partial
constexpr int kSub = 128;          // rows staged in LDS at a time

int corr_chunks(int64_t N) { return (int)((N + kChunkRows - 1) / kChunkRows); }
int corr_rpad(int r) { return (r + 31) / 32 * 32; }

// grid (chunks, ceil(b/32), rpad/32), 256 threads = 4 wavefronts; each
// wavefront covers a quarter of each staged slice and every lane a 4 x 4
// block of the 32 x 32 tile (j = 4 (lane/8) + i, s = 4 (lane%8) + k).
__global__ __launch_bounds__(256) void k_corr_partial(const float *__restrict__ x, int64_t ldx, int N, int b,
                                                      const float *__restrict__ U, int64_t ldu, int r,
                                                      float *__restrict__ part, int rpad) {
  __shared__ float sm[2 * 32 * (kSub + 1)];
  float(*Us)[kSub + 1] = reinterpret_cast<float(*)[kSub + 1]>(sm);
  float(*Xs)[kSub + 1] = reinterpret_cast<float(*)[kSub + 1]>(sm + 32 * (kSub + 1));
  const int chunk = blockIdx.x;
  const int s_base = blockIdx.y * 32, j_base = blockIdx.z * 32;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int jq = lane >> 3, sq = lane & 7;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[i][k] = 0.f;
  const int n_chunk = chunk * kChunkRows;
  for (int sub = 0; sub < kChunkRows; sub += kSub) {
    const int n0 = n_chunk + sub;
    if (n0 >= N) break;
    for (int e = threadIdx.x; e < 32 * kSub; e += 256) {
      const int jj = e / kSub, nn = e % kSub;
      const int n = n0 + nn;
      const int j = j_base + jj, s = s_base + jj;
      Us[jj][nn] = (n < N && j < r) ? U[(int64_t)j * ldu + n] : 0.f;
      Xs[jj][nn] = (n < N && s < b) ? x[(int64_t)s * ldx + n] : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < kSub / 4; ++rr) {
      const int nn = wave * (kSub / 4) + rr;
      float u[4], v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        u[i] = Us[jq * 4 + i][nn];
        v[i] = Xs[sq * 4 + i][nn];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[i][k] += u[i] * v[k];
    }
    __syncthreads();
  }
  float *red = sm;  // 4 x 1024 floats
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) red[wave * 1024 + (jq * 4 + i) * 32 + sq * 4 + k] = acc[i][k];
  __syncthreads();
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const float v = (red[e] + red[1024 + e]) + (red[2048 + e] + red[3072 + e]);
    const int j = j_base + e / 32, s = s_base + e % 32;
    if (j < r && s < b) part[((int64_t)chunk * rpad + j) * b + s] = v;
  }
}

hipError_t corr_partial(const float *x, int64_t ldx, int64_t N, int64_t b, const float *U, int64_t ldu, int r,
                        float *part, hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  if (b > 32 * 65535 || r > 32 * 65535) return hipErrorInvalidValue;
  const int rpad = corr_rpad(r);
  const dim3 grid(corr_chunks(N), (unsigned)((b + 31) / 32), rpad / 32);
  SLP_LAUNCH("corr_partial", k_corr_partial, grid, dim3(256), 0, st, x, ldx, (int)N, (int)b, U, ldu, r, part, rpad);
  return hipGetLastError();
}

__global__ void k_corr_reduce(const float *__restrict__ part, int chunks, int rpad, int b, int r,
                              const float *__restrict__ d, float *__restrict__ dC) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)b * r) return;
  const int s = (int)(idx / r), j = (int)(idx % r);
  float acc = 0.f;
  for (int c = 0; c < chunks; ++c) acc += part[((int64_t)c * rpad + j) * b + s];
  dC[(int64_t)s * rpad + j] = d[j] * acc;
}

hipError_t corr_reduce(const float *part, int64_t N, int64_t b, int r, const float *d, float *dC, hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  const int64_t tot = b * r;
  SLP_LAUNCH("corr_reduce", k_corr_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, part, corr_chunks(N),
                     corr_rpad(r), (int)b, r, d, dC);
  return hipGetLastError();
}

// c[s * ldc + j] = sum_chunk part[chunk][j][s] (coefficients S_K^T x).
__global__ void k_corr_sum(const float *__restrict__ part, int chunks, int rpad, int b, int r,
                           float *__restrict__ c, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)b * r) return;
  const int s = (int)(idx / r), j = (int)(idx % r);
  float acc = 0.f;
  for (int q = 0; q < chunks; ++q) acc += part[((int64_t)q * rpad + j) * b + s];
  c[(int64_t)s * ldc + j] = acc;
}

hipError_t corr_sum(const float *part, int64_t N, int64_t b, int r, float *c, int64_t ldc, hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  const int64_t tot = b * r;
  SLP_LAUNCH("corr_sum", k_corr_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, part, corr_chunks(N),
                     corr_rpad(r), (int)b, r, c, ldc);
  return hipGetLastError();
}

// y[s][n] += sum_j U[n,j] dC[s][j]: one row per lane, 64 signals per
// workgroup, the U row held in registers 64 columns at a time.
constexpr int kApplySig = 64;
__global__ __launch_bounds__(256) void k_corr_apply(float *__restrict__ y, int64_t ldy, int N, int b,
                                                    const float *__restrict__ U, int64_t ldu, int r,
                                                    const float *__restrict__ dC, int rpad) {
  __shared__ float dcs[kApplySig][65];
  const int n = blockIdx.x * 256 + threadIdx.x;
  const int s_base = blockIdx.y * kApplySig;
  for (int j0 = 0; j0 < r; j0 += 64) {
    const int jn = r - j0 < 64 ? r - j0 : 64;
    __syncthreads();
    for (int e = threadIdx.x; e < kApplySig * 64; e += 256) {
      const int ss = e / 64, jj = e % 64;
      const int s = s_base + ss;
      dcs[ss][jj] = (s < b && jj < jn) ? dC[(int64_t)s * rpad + j0 + jj] : 0.f;
    }
    __syncthreads();
    if (n < N) {
      float u[64];
#pragma unroll
      for (int jj = 0; jj < 64; ++jj) u[jj] = jj < jn ? U[(int64_t)(j0 + jj) * ldu + n] : 0.f;
      const int sn = b - s_base < kApplySig ? b - s_base : kApplySig;
      for (int ss = 0; ss < sn; ++ss) {
        float acc = 0.f;
#pragma unroll
        for (int jj = 0; jj < 64; ++jj) acc += u[jj] * dcs[ss][jj];
        y[(int64_t)(s_base + ss) * ldy + n] += acc;
      }
    }
  }
}

hipError_t corr_apply(float *y, int64_t ldy, int64_t N, int64_t b, const float *U, int64_t ldu, int r,
                      const float *dC, hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  const dim3 grid((unsigned)((N + 255) / 256), (unsigned)((b + kApplySig - 1) / kApplySig));
  SLP_LAUNCH("corr_apply", k_corr_apply, grid, dim3(256), 0, st, y, ldy, (int)N, (int)b, U, ldu, r, dC, corr_rpad(r));
  return hipGetLastError();
}

}  // namespace slp

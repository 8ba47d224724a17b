// FP64 setup kernels: the Slepian vectors of the transition region.
//
// The paper precomputes the Slepian vectors whose eigenvalues lie in
// (eps, 1 - eps) (Section 1.3, "fast precomputation"; Section 4.1) and cites
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
#include <vector>

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
// The quotient e2/q uses the hardware reciprocal refined by two Newton steps
// (a few ulp, far inside the perturbation the count tolerates; the |q| >=
// pivmin guard keeps it away from zero), and T's entries are read eight at a
// time ahead of the recurrence.
__device__ __forceinline__ double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

__device__ __forceinline__ int sturm_count(const double *__restrict__ a, const double *__restrict__ e2,
                                           int64_t N, double x, double pivmin) {
  double q = a[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  int64_t k = 1;
  for (; k + 8 <= N; k += 8) {
    double av[8], ev[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      av[i] = a[k + i];
      ev[i] = e2[k - 1 + i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      q = (av[i] - x) - ev[i] * recip(q);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
  }
  for (; k < N; ++k) {
    q = (a[k] - x) - e2[k - 1] * recip(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// One workgroup per eigenvalue theta_t (ascending index t): keep
// [lo, hi) with count(lo) <= t < count(hi) and split it at blockDim.x points
// per round until it is as narrow as FP64 allows.
__device__ __forceinline__ void bisect_body(const double *__restrict__ a, const double *__restrict__ e2, int64_t N,
                                            double gl, double gu, double pivmin, double atol, int64_t t,
                                            double *__restrict__ theta_t) {
  __shared__ int first;
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
  if (threadIdx.x == 0) *theta_t = 0.5 * (lo + hi);
}

__global__ __launch_bounds__(256) void k_bisect(const double *__restrict__ a, const double *__restrict__ e2,
                                                int64_t N, double gl, double gu, double pivmin, double atol,
                                                int64_t t0, double *__restrict__ theta) {
  bisect_body(a, e2, N, gl, gu, pivmin, atol, t0 + blockIdx.x, theta + blockIdx.x);
}

hipError_t tridiag_bisect(const double *a, const double *e2, int64_t N, double gl, double gu, double pivmin,
                          int64_t t0, int64_t count, double *theta, hipStream_t st) {
  const double atol = DBL_EPSILON * fmax(fabs(gl), fabs(gu));
  hipLaunchKernelGGL(k_bisect, dim3((unsigned)count), dim3(256), 0, st, a, e2, N, gl, gu, pivmin, atol, t0,
                     theta);
  return hipGetLastError();
}

// Scratch of inverse iteration, interleaved [k][vector] so that the lanes of
// a wavefront (one vector each) touch consecutive addresses: the iterate x,
// the reciprocal pivots of U, U's first superdiagonal and the row-exchange
// flags (U's second superdiagonal is off[k+1] after an exchange, else zero,
// so it is not stored).
struct InvScratch {
  double *x, *dinv, *du;
  unsigned char *piv;
};

static InvScratch carve(void *p, int64_t N, int64_t count) {
  InvScratch s;
  const size_t nd = (size_t)N * (size_t)count;
  double *q = (double *)p;
  s.x = q;
  s.dinv = q + nd;
  s.du = q + 2 * nd;
  s.piv = (unsigned char *)(q + 3 * nd);
  return s;
}

size_t inviter_scratch_bytes(int64_t N, int64_t count) {
  return (size_t)N * (size_t)count * (3 * sizeof(double) + 1) + 256;
}

__device__ __forceinline__ double start_value(int64_t k, int64_t j) {
  uint32_t h = (uint32_t)(k * 2654435761ull) ^ (uint32_t)(j * 40503u + 0x9e3779b9u);
  h ^= h >> 16;
  h *= 0x7feb352du;
  h ^= h >> 15;
  return 0.5 + (double)(h & 0xffffu) / 65536.0;
}

// Steps of the sequential sweeps whose operands are fetched one block ahead
// of the arithmetic, so each lane's chain waits on memory once per block.
constexpr int kIB = 8;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Raw buffer access: one per-lane byte offset (the lane's column) and one
// uniform byte offset (the row), so a step's four accesses share their
// address arithmetic, which runs on the scalar unit.  Reads past num_records
// return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, int64_t bytes) {
  const int n = bytes > 0x7fffffff ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, n, 0x00020000);
}
__device__ __forceinline__ double bld(__amdgpu_buffer_rsrc_t r, int vo, int so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
__device__ __forceinline__ void bst(double v, __amdgpu_buffer_rsrc_t r, int vo, int so) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, 0);
}

// One lane per eigenvalue: `iters` rounds of x <- (T - theta I)^{-1} x with
// normalisation.  Each round factors T - theta I = P L U on the fly
// (Gaussian elimination with partial pivoting, LAPACK's choice for inverse
// iteration on a tridiagonal matrix), applying each multiplier of L to the
// iterate as it is produced, and stores what the backward substitution with
// U needs.  The first round starts from a hashed vector.  The final
// (unnormalised) iterate is left in s.x.  Rows of the scratch arrays are
// addressed from a base that moves with the block, so no offset exceeds a
// block's span.
__device__ __forceinline__ void inviter_body(const double *__restrict__ a, const double *__restrict__ off,
                                             int64_t N, const double *__restrict__ theta, int64_t count,
                                             InvScratch s, double tiny, int iters, int64_t j) {
  if (j >= count) return;
  const double th = theta[j];
  const int64_t C = count;
  if (N == 1) {
    s.x[j] = 1.0;
    return;
  }
  const int64_t M = N - 1;  // elimination steps k = 0..N-2; off[k] valid for k < M
  const int rs8 = (int)(C * 8), rs1 = (int)C;  // row strides in bytes (kIB rows stay far below 2^31)
  const int vo8 = (int)j * 8, vo1 = (int)j;
  // T's entries are the same for every lane; a per-lane byte offset keeps
  // the prefetched blocks in vector registers.
  const int tz = (int)__builtin_amdgcn_mbcnt_lo(0u, 0u) * 8;
  const __amdgpu_buffer_rsrc_t ra = rsrc(a, N * 8), ro = rsrc(off, M * 8);
  auto rows = [&](int64_t r0, __amdgpu_buffer_rsrc_t &rx, __amdgpu_buffer_rsrc_t &rd, __amdgpu_buffer_rsrc_t &ru,
                  __amdgpu_buffer_rsrc_t &rp) {
    const int64_t o = r0 * C, n = (N - r0) * C;
    rx = rsrc(s.x + o, n * 8);
    rd = rsrc(s.dinv + o, n * 8);
    ru = rsrc(s.du + o, n * 8);
    rp = rsrc(s.piv + o, n);
  };
  double scale = 1.0;
  for (int it = 0; it < iters; ++it) {
    // ---- forward: elimination with the multipliers applied to x ----
    double cur_d = bld(ra, tz, 0) - th;
    double cur_du = bld(ro, tz, 0);
    double prev = it == 0 ? start_value(0, j) : s.x[j] * scale;
    // block k0: x[k+1], a[k+1], off[k] for k = k0..k0+kIB-1, and off[k0+kIB]
    auto load_fwd = [&](int64_t k0, double (&bx)[kIB], double (&ba)[kIB], double (&bo)[kIB + 1]) {
      __amdgpu_buffer_rsrc_t rx, rd, ru, rp;
      rows(k0 + 1 < N ? k0 + 1 : M, rx, rd, ru, rp);
#pragma unroll
      for (int i = 0; i < kIB; ++i) {
        const int64_t k = k0 + i;
        bx[i] = it == 0 ? start_value(k + 1, j) : bld(rx, vo8, i * rs8);
        ba[i] = bld(ra, tz, (int)((k + 1) * 8));
        bo[i] = bld(ro, tz, (int)(k * 8));
      }
      bo[kIB] = bld(ro, tz, (int)((k0 + kIB) * 8));
    };
    double cx[kIB], ca[kIB], co[kIB + 1];
    load_fwd(0, cx, ca, co);
    for (int64_t k0 = 0; k0 < M; k0 += kIB) {
      const bool more = k0 + kIB < M;
      double nx[kIB], na[kIB], no[kIB + 1];
      if (more) load_fwd(k0 + kIB, nx, na, no);
      __amdgpu_buffer_rsrc_t rx, rd, ru, rp;
      rows(k0, rx, rd, ru, rp);
#pragma unroll
      for (int i = 0; i < kIB; ++i) {
        const int64_t k = k0 + i;
        if (k >= M) break;  // uniform
        const double sub = co[i];
        const double nd = ca[i] - th;
        const double nu = k + 1 < M ? co[i + 1] : 0.0;
        const double nxt = cx[i] * scale;
        const bool sw = fabs(cur_d) < fabs(sub);  // exchange rows k and k+1
        const double pv = sw ? sub : (cur_d == 0.0 ? tiny : cur_d);
        const double rk = 1.0 / pv;
        const double f = (sw ? cur_d : sub) * rk;
        bst(rk, rd, vo8, i * rs8);
        bst(sw ? nd : cur_du, ru, vo8, i * rs8);
        __builtin_amdgcn_raw_buffer_store_b8((unsigned char)(sw ? 1 : 0), rp, vo1, i * rs1, 0);
        bst(sw ? nxt : prev, rx, vo8, i * rs8);
        prev = sw ? prev - f * nxt : nxt - f * prev;
        const double ncd = sw ? cur_du - f * nd : nd - f * cur_du;
        cur_du = sw ? -f * nu : nu;
        cur_d = ncd;
      }
      if (more) {
#pragma unroll
        for (int i = 0; i < kIB; ++i) {
          cx[i] = nx[i];
          ca[i] = na[i];
          co[i] = no[i];
        }
        co[kIB] = no[kIB];
      }
    }
    s.dinv[M * C + j] = 1.0 / (cur_d == 0.0 ? tiny : cur_d);
    s.x[M * C + j] = prev;
    // ---- backward substitution with U, k = N-1 .. 0 ----
    // block k0: rows k0, k0-1, .., k0-kIB+1 (x, 1/u_kk, u_k,k+1, flag, off[k+1]),
    // addressed from row max(k0 - kIB + 1, 0)
    auto load_bwd = [&](int64_t k0, double (&bx)[kIB], double (&bd)[kIB], double (&bu)[kIB],
                        unsigned char (&bp)[kIB], double (&bo)[kIB]) {
      const int64_t r0 = k0 - kIB + 1 > 0 ? k0 - kIB + 1 : 0;
      __amdgpu_buffer_rsrc_t rx, rd, ru, rp;
      rows(r0, rx, rd, ru, rp);
#pragma unroll
      for (int i = 0; i < kIB; ++i) {
        const int64_t k = k0 - i >= 0 ? k0 - i : 0;
        const int q = (int)(k - r0);
        bx[i] = bld(rx, vo8, q * rs8);
        bd[i] = bld(rd, vo8, q * rs8);
        bu[i] = k < M ? bld(ru, vo8, q * rs8) : 0.0;
        bp[i] = k < M ? __builtin_amdgcn_raw_buffer_load_b8(rp, vo1, q * rs1, 0) : 0;
        bo[i] = k + 1 < M ? bld(ro, tz, (int)((k + 1) * 8)) : 0.0;
      }
    };
    double x1 = 0.0, x2 = 0.0, ss = 0.0;
    double rxv[kIB], rdv[kIB], ruv[kIB], rov[kIB];
    unsigned char rpv[kIB];
    load_bwd(M, rxv, rdv, ruv, rpv, rov);
    for (int64_t k0 = M; k0 >= 0; k0 -= kIB) {
      const bool more = k0 - kIB >= 0;
      double nx[kIB], nd[kIB], nu[kIB], no[kIB];
      unsigned char np[kIB];
      if (more) load_bwd(k0 - kIB, nx, nd, nu, np, no);
      const int64_t r0 = k0 - kIB + 1 > 0 ? k0 - kIB + 1 : 0;
      __amdgpu_buffer_rsrc_t rx, rd, ru, rp;
      rows(r0, rx, rd, ru, rp);
#pragma unroll
      for (int i = 0; i < kIB; ++i) {
        const int64_t k = k0 - i;
        if (k < 0) break;  // uniform
        double v = rxv[i] - ruv[i] * x1;
        if (rpv[i]) v -= rov[i] * x2;
        v *= rdv[i];
        bst(v, rx, vo8, (int)(k - r0) * rs8);
        ss += v * v;
        x2 = x1;
        x1 = v;
      }
      if (more) {
#pragma unroll
        for (int i = 0; i < kIB; ++i) {
          rxv[i] = nx[i];
          rdv[i] = nd[i];
          ruv[i] = nu[i];
          rpv[i] = np[i];
          rov[i] = no[i];
        }
      }
    }
    scale = 1.0 / sqrt(ss);
  }
}

__global__ __launch_bounds__(64) void k_inviter(const double *__restrict__ a, const double *__restrict__ off,
                                                int64_t N, const double *__restrict__ theta, int64_t count,
                                                InvScratch s, double tiny, int iters) {
  inviter_body(a, off, N, theta, count, s, tiny, iters, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Normalise to unit 2-norm, sign so that the first entry of magnitude
// >= 1e-3 max|v| is positive, and write column count-1-j of V.
__device__ __forceinline__ void normalize_body(InvScratch s, int64_t N, int64_t count, double *__restrict__ V,
                                               int64_t j) {
  __shared__ double red[256];
  __shared__ int64_t redi[256];
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

__global__ __launch_bounds__(256) void k_normalize(InvScratch s, int64_t N, int64_t count, double *__restrict__ V) {
  normalize_body(s, N, count, V, blockIdx.x);
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

// ---- many plans in one launch ----
// Workgroup w belongs to job q with start[q] <= w < start[q + 1] (binary
// search), and runs the same body as the one-plan kernels on that job's
// operands, so a plan's vectors do not depend on the company it is solved in.

struct EigJobDev {
  const double *a, *e2, *off;
  int64_t N, t0, count;
  double gl, gu, pivmin, atol, tiny;
  double *theta, *V;
  InvScratch s;
};

__device__ __forceinline__ int job_of(const int *__restrict__ start, int m, int w) {
  int lo = 0, hi = m;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= w) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_bisect_many(const EigJobDev *__restrict__ jobs, const int *__restrict__ start,
                                                     int m) {
  const int q = job_of(start, m, blockIdx.x);
  const EigJobDev &J = jobs[q];
  const int64_t i = (int64_t)blockIdx.x - start[q];
  bisect_body(J.a, J.e2, J.N, J.gl, J.gu, J.pivmin, J.atol, J.t0 + i, J.theta + i);
}

__global__ __launch_bounds__(64) void k_inviter_many(const EigJobDev *__restrict__ jobs, const int *__restrict__ start,
                                                     int m, int iters) {
  const int q = job_of(start, m, blockIdx.x);
  const EigJobDev &J = jobs[q];
  const int64_t j = ((int64_t)blockIdx.x - start[q]) * 64 + threadIdx.x;
  inviter_body(J.a, J.off, J.N, J.theta, J.count, J.s, J.tiny, iters, j);
}

__global__ __launch_bounds__(256) void k_normalize_many(const EigJobDev *__restrict__ jobs,
                                                        const int *__restrict__ start, int m) {
  const int q = job_of(start, m, blockIdx.x);
  const EigJobDev &J = jobs[q];
  normalize_body(J.s, J.N, J.count, J.V, (int64_t)blockIdx.x - start[q]);
}

hipError_t eig_solve_many(const EigJob *jobs, int m, int iters, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  std::vector<EigJobDev> dj(m);
  std::vector<int> sb(m + 1), si(m + 1);
  sb[0] = si[0] = 0;
  for (int q = 0; q < m; ++q) {
    const EigJob &J = jobs[q];
    EigJobDev &d = dj[q];
    d.a = J.a;
    d.e2 = J.e2;
    d.off = J.off;
    d.N = J.N;
    d.t0 = J.t0;
    d.count = J.count;
    d.gl = J.gl;
    d.gu = J.gu;
    d.pivmin = J.pivmin;
    d.atol = DBL_EPSILON * fmax(fabs(J.gl), fabs(J.gu));
    d.tiny = DBL_EPSILON * 0.25 * (double)J.N * (double)J.N;
    d.theta = J.theta;
    d.V = J.V;
    d.s = carve(J.scratch, J.N, J.count);
    if ((int64_t)sb[q] + J.count > 0x7fffffff) return hipErrorInvalidValue;
    sb[q + 1] = sb[q] + (int)J.count;
    si[q + 1] = si[q] + (int)((J.count + 63) / 64);
  }
  EigJobDev *djd = nullptr;
  int *sd = nullptr;
  hipError_t e = hipMalloc(&djd, m * sizeof(EigJobDev));
  if (e != hipSuccess) return e;
  e = hipMalloc(&sd, 2 * (m + 1) * sizeof(int));
  if (e != hipSuccess) {
    (void)hipFree(djd);
    return e;
  }
  e = hipMemcpyAsync(djd, dj.data(), m * sizeof(EigJobDev), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(sd, sb.data(), (m + 1) * sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(sd + m + 1, si.data(), (m + 1) * sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_bisect_many, dim3((unsigned)sb[m]), dim3(256), 0, st, djd, sd, m);
    hipLaunchKernelGGL(k_inviter_many, dim3((unsigned)si[m]), dim3(64), 0, st, djd, sd + m + 1, m, iters);
    hipLaunchKernelGGL(k_normalize_many, dim3((unsigned)sb[m]), dim3(256), 0, st, djd, sd, m);
    e = hipGetLastError();
  }
  const hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(djd);
  (void)hipFree(sd);
  return e != hipSuccess ? e : e2;
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

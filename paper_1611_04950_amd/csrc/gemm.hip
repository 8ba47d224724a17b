// Slepian coefficients c = S_K^T x (Section 1.3, the compression S_K^* x) as a
// plain library GEMM on the matrix cores.  S_K is N x K column-major (every
// Slepian vector contiguous) and x is N x b column-major, so both operands
// run along the reduction index n:
//   mode 0  one FP32 GEMM;
//   mode 1  BF16 hi/lo halves of both operands (v = hi + lo, hi = bf16(v),
//           lo = bf16(v - hi)), three GEMMs hi*hi + hi*lo + lo*hi into one
//           FP32 result, accumulated in that fixed order.
// The GEMMs are hipBLASLt's; the algorithm the library's heuristic picks for a
// shape is kept by the caller's cache so that repeated calls reuse it.
#include <hipblaslt/hipblaslt.h>

#include <cstring>
#include <map>
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// hi/lo halves of an N x b FP32 matrix (leading dimension ld_src) into BF16
// planes with leading dimension ld (rows N..ld-1 untouched).  Two columns'
// worth of rows per thread pair: thread (n, s) with n even handles n, n + 1.
__global__ __launch_bounds__(256) void k_split_bf16(const float *__restrict__ x, int64_t ldx, int64_t N,
                                                    __bf16 *__restrict__ hi, __bf16 *__restrict__ lo, int64_t ld) {
  const int64_t n = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
  const int64_t s = blockIdx.y;
  if (n >= N) return;
  const float *xs = x + s * ldx;
  const f32x2 a = {xs[n], n + 1 < N ? xs[n + 1] : 0.f};
  const bf16x2 h = __builtin_convertvector(a, bf16x2);
  const bf16x2 l = __builtin_convertvector(a - __builtin_convertvector(h, f32x2), bf16x2);
  hi[s * ld + n] = h[0];
  lo[s * ld + n] = l[0];
  if (n + 1 < N) {
    hi[s * ld + n + 1] = h[1];
    lo[s * ld + n + 1] = l[1];
  }
}

hipError_t split_bf16(const float *x, int64_t ldx, int64_t N, int64_t b, __bf16 *hi, __bf16 *lo, int64_t ld,
                      hipStream_t st) {
  if (N == 0 || b == 0) return hipSuccess;
  if (b > 65535) return hipErrorInvalidValue;
  SLP_LAUNCH("split_bf16", k_split_bf16, dim3((unsigned)((N + 511) / 512), (unsigned)b), dim3(256), 0, st, x, ldx,
             N, hi, lo, ld);
  return hipGetLastError();
}

// dst (rows x cols, ldd) = src (lds), FP32
__global__ __launch_bounds__(256) void k_copy_f32(const float *__restrict__ src, int64_t lds, float *__restrict__ dst,
                                                  int64_t ldd, int64_t rows) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r < rows) dst[c * ldd + r] = src[c * lds + r];
}

hipError_t copy_f32(const float *src, int64_t lds, float *dst, int64_t ldd, int64_t rows, int64_t cols,
                    hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  if (cols > 65535) return hipErrorInvalidValue;
  SLP_LAUNCH("copy_f32", k_copy_f32, dim3((unsigned)((rows + 255) / 256), (unsigned)cols), dim3(256), 0, st, src,
             lds, dst, ldd, rows);
  return hipGetLastError();
}

namespace {
std::mutex g_lt_mu;
std::map<int, hipblasLtHandle_t> g_lt;  // one handle per device, kept until the process ends

hipblasLtHandle_t lt_handle(int device) {
  std::lock_guard<std::mutex> lock(g_lt_mu);
  auto it = g_lt.find(device);
  if (it != g_lt.end()) return it->second;
  hipblasLtHandle_t h = nullptr;
  if (hipblasLtCreate(&h) != HIPBLAS_STATUS_SUCCESS) return nullptr;
  g_lt[device] = h;
  return h;
}

// Descriptors of one GEMM C (K x b) = A^T B, A: N x K (lda), B: N x b (ldb).
struct Lt {
  hipblasLtMatmulDesc_t op = nullptr;
  hipblasLtMatrixLayout_t a = nullptr, b = nullptr, c = nullptr;
  ~Lt() {
    if (op) hipblasLtMatmulDescDestroy(op);
    if (a) hipblasLtMatrixLayoutDestroy(a);
    if (b) hipblasLtMatrixLayoutDestroy(b);
    if (c) hipblasLtMatrixLayoutDestroy(c);
  }
  bool make(hipDataType in, int64_t N, int64_t K, int64_t nb, int64_t lda, int64_t ldb, int64_t ldc) {
    if (hipblasLtMatmulDescCreate(&op, HIPBLAS_COMPUTE_32F, HIP_R_32F) != HIPBLAS_STATUS_SUCCESS) return false;
    const int32_t ta = HIPBLAS_OP_T, tb = HIPBLAS_OP_N;
    if (hipblasLtMatmulDescSetAttribute(op, HIPBLASLT_MATMUL_DESC_TRANSA, &ta, sizeof(ta)) != HIPBLAS_STATUS_SUCCESS)
      return false;
    if (hipblasLtMatmulDescSetAttribute(op, HIPBLASLT_MATMUL_DESC_TRANSB, &tb, sizeof(tb)) != HIPBLAS_STATUS_SUCCESS)
      return false;
    return hipblasLtMatrixLayoutCreate(&a, in, (uint64_t)N, (uint64_t)K, lda) == HIPBLAS_STATUS_SUCCESS &&
           hipblasLtMatrixLayoutCreate(&b, in, (uint64_t)N, (uint64_t)nb, ldb) == HIPBLAS_STATUS_SUCCESS &&
           hipblasLtMatrixLayoutCreate(&c, HIP_R_32F, (uint64_t)K, (uint64_t)nb, ldc) == HIPBLAS_STATUS_SUCCESS;
  }
};
}  // namespace

int coeffs_gemm(int device, int mode, const void *S, const void *Slo, int64_t lds, const void *X, const void *Xlo,
                int64_t ldx, float *c, int64_t ldc, int64_t N, int64_t K, int64_t b, void *ws, size_t ws_bytes,
                GemmCache &cache, hipStream_t st) {
  hipblasLtHandle_t h = lt_handle(device);
  if (!h) return -1;
  Lt d;
  if (!d.make(mode == 0 ? HIP_R_32F : HIP_R_16BF, N, K, b, lds, ldx, ldc)) return -1;
  const bool hit = cache.valid && cache.mode == mode && cache.N == N && cache.K == K && cache.b == b &&
                   cache.lds == lds && cache.ldx == ldx && cache.ldc == ldc && cache.ws_max == ws_bytes;
  if (!hit) {
    hipblasLtMatmulPreference_t pref = nullptr;
    if (hipblasLtMatmulPreferenceCreate(&pref) != HIPBLAS_STATUS_SUCCESS) return -1;
    const uint64_t wmax = ws_bytes;
    hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wmax, sizeof(wmax));
    hipblasLtMatmulHeuristicResult_t res[1];
    int got = 0;
    const hipblasStatus_t hs = hipblasLtMatmulAlgoGetHeuristic(h, d.op, d.a, d.b, d.c, d.c, pref, 1, res, &got);
    hipblasLtMatmulPreferenceDestroy(pref);
    if (hs != HIPBLAS_STATUS_SUCCESS || got < 1 || res[0].state != HIPBLAS_STATUS_SUCCESS) return -2;
    static_assert(sizeof(hipblasLtMatmulAlgo_t) <= sizeof(cache.algo), "algorithm record");
    std::memcpy(cache.algo, &res[0].algo, sizeof(hipblasLtMatmulAlgo_t));
    cache.ws = res[0].workspaceSize;
    cache.mode = mode;
    cache.N = N;
    cache.K = K;
    cache.b = b;
    cache.lds = lds;
    cache.ldx = ldx;
    cache.ldc = ldc;
    cache.ws_max = ws_bytes;
    cache.valid = true;
  }
  const float one = 1.0f, zero = 0.0f;
  auto run = [&](const void *A, const void *B, const float *beta) {
    return hipblasLtMatmul(h, d.op, &one, A, d.a, B, d.b, beta, c, d.c, c, d.c,
                           reinterpret_cast<const hipblasLtMatmulAlgo_t *>(cache.algo), ws, cache.ws, st);
  };
  const bool tr = trace_enabled();
  if (tr) trace_mark_begin(mode == 0 ? "coeffs_gemm" : "coeffs_gemm_bf16x3", st);
  hipblasStatus_t s = run(S, X, &zero);
  if (s == HIPBLAS_STATUS_SUCCESS && mode != 0) s = run(S, Xlo, &one);
  if (s == HIPBLAS_STATUS_SUCCESS && mode != 0) s = run(Slo, X, &one);
  if (tr) trace_mark_end(st);
  return s == HIPBLAS_STATUS_SUCCESS ? 0 : -1;
}

}  // namespace slp

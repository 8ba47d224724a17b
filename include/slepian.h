/*
 * slepian.h -- C ABI of libslepian, a gfx950 (MI355X) implementation of the
 * fast Slepian transform of Karnik, Zhu, Wakin, Romberg and Davenport
 * ("The Fast Slepian Transform", arXiv:1611.04950).
 *
 * Notation (Sections 1.1-1.2 of the paper): N signal length, W in (0, 1/2)
 * half bandwidth, B the N x N prolate matrix B[m,n] = sin(2 pi W (m-n)) /
 * (pi (m-n)) (diagonal 2W), lambda_0 > ... > lambda_{N-1} its eigenvalues,
 * S = [s_0 ... s_{N-1}] its orthonormal eigenvectors (the Slepian basis),
 * S_K the first K columns, eps in (0, 1/2) the tolerance of the fast
 * operators.  K defaults to round(2NW) with halves rounded away from zero
 * (Section 4.1).
 *
 * Conventions shared by every call:
 *   - Signals are real.  A batch of b signals of length N is column-major
 *     N x b: signal s starts at x + s*ldx, ldx >= N.  All signal, output and
 *     workspace pointers are DEVICE pointers on the plan's device, owned by
 *     the caller; host pointers are marked "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls enqueue work on `stream` and return without synchronising unless
 *     stated otherwise.  A plan does not change after creation except for
 *     buffers built on first use and then kept (the Slepian vectors of
 *     slepian_coeffs, U's layouts for band sets), which are built under a
 *     lock; concurrent calls on different streams need separate workspaces.
 *   - Workspace: pass work = NULL, work_bytes = 0 to let the plan use an
 *     internal buffer (grown on demand; then calls on one plan must not run
 *     concurrently), or pass a buffer of at least slepian_workspace_size()
 *     bytes.
 *   - Errors: every call returns SLEPIAN_OK (0) or a negative status.  All
 *     argument checks happen before anything is enqueued, so a failed call
 *     leaves outputs untouched.  Calls never abort the process.
 */
#ifndef SLEPIAN_H_
#define SLEPIAN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slepian_plan_s *slepian_plan_t;
typedef struct slepian_group_s *slepian_group_t;
typedef struct slepian_bands_s *slepian_bands_t;

enum slepian_status {
  SLEPIAN_OK = 0,
  SLEPIAN_EINVAL = -1,     /* argument outside its domain (N < 2, W not in (0,1/2),
                              eps not in (0,1/2), alpha <= 0, ld < N, batch < 0, ...) */
  SLEPIAN_EGAP = -2,       /* K violates lambda_{K-1} > eps and lambda_K < 1 - eps
                              (Corollary 2's condition on K) */
  SLEPIAN_ENOMEM = -3,     /* device or host allocation failed, or workspace too small */
  SLEPIAN_EHIP = -4,       /* a HIP runtime call failed */
  SLEPIAN_ENOCONV = -5,    /* eigensolver check or iterative refinement did not converge */
  SLEPIAN_ENOTSUP = -6,    /* size or mode the library does not support  */
  SLEPIAN_ENONFINITE = -7, /* NaN or Inf in the input, seen by the synchronous iterative calls
                              (slepian_lsq when it computes residuals, slepian_project_bands_span)
                              as a non-finite norm; the asynchronous calls do not check */
  SLEPIAN_EIO = -8,        /* plan file could not be read or written, or is malformed */
  SLEPIAN_ESCRATCH = -9,   /* slepian_project_noalloc: two signals need more than its fixed scratch */
  SLEPIAN_EINTERNAL = -10  /* unexpected internal failure (a bug; please report) */
};

/* Arithmetic of the low-rank correction (the B x product is always FP32). */
enum slepian_precision {
  SLEPIAN_FP32 = 0,        /* FP32 correction */
  SLEPIAN_MIXED = 1,       /* BF16 hi/lo split on matrix cores, FP32 accumulation */
  SLEPIAN_BF16_RAW = 2     /* BF16 operands only (no lo terms); for error studies */
};

enum slepian_lsq_mode {
  SLEPIAN_PINV = 0,        /* rank-K truncated pseudoinverse of B (Corollary 3) */
  SLEPIAN_TIKHONOV = 1     /* (B^2 + alpha I)^{-1} B (Corollary 4) */
};

enum slepian_op {
  SLEPIAN_OP_PROJECT = 0,
  SLEPIAN_OP_COEFFS = 1,
  SLEPIAN_OP_LSQ = 2,
  SLEPIAN_OP_MULTIBAND = 3  /* batch argument of slepian_workspace_size = bands x signals */
};

typedef struct {
  double alpha;     /* > 0: also prepare the Tikhonov set for this alpha (Lemma 6); 0: none */
  int64_t K;        /* 0: K = round(2NW); else 1 <= K <= N-1 */
  int precision;    /* enum slepian_precision used by slepian_project */
  int device;       /* HIP device ordinal, -1: the current device */
  int tune;         /* 1: choose the product's launch variants by timing at creation (three-pass
                       plans: rows of 2^13 or 2^12 points, the update fused into the inverse
                       column pass up to L1 = 16 or 32, that pass's workgroup shape); 2: the
                       same among the variants groups launch together (L1 <= 32); 0: defaults.
                       The variants split the work differently, not the arithmetic: results stay
                       within FP32 rounding of the untuned plan's, and a group reproduces a tuned
                       plan's own calls bit for bit. */
  int64_t tune_batch;     /* signals to time with (0: 64); the choice is for batches of this size */
  const char *tune_cache; /* host path of a text tuning cache, or NULL: a choice recorded there for
                             the same (N, W, eps, precision, tune_batch) is reused without timing,
                             and a new one is appended.  Unreadable or malformed lines are skipped. */
} slepian_plan_opts;

typedef struct {
  int64_t N;
  double W, eps, alpha;
  int64_t K;
  int64_t L;            /* FFT length used for B x: smallest power of two >= 2N */
  int64_t r;            /* |I2 u I3| = #{eps < lambda < 1-eps} (Lemma 4) */
  int64_t l_first;      /* index l of the first transition vector */
  int64_t r_tik;        /* #{alpha(1+alpha)eps < lambda < 1-eps/3} (Lemma 6), 0 if alpha == 0 */
  int64_t l_first_tik;
  int64_t window_lo, window_hi;  /* eigen-indices solved at setup (inclusive) */
  double lam_Km1, lam_K;         /* lambda_{K-1}, lambda_K */
  double eps_achieved;  /* max(1 - lambda over I1, lambda over I4) seen at the window edges,
                           an upper bound on ||S_K S_K^T - (B + U diag(d) U^T)|| (Lemma 4) */
  int precision;
  int device;
  int32_t row_log2;     /* FP32 product: log2 of its row transform length (L for a single pass) */
  int32_t col_log2;     /* FP32 product: log2 L1 of its column transforms (0: single pass) */
  int32_t cic_shape;    /* tuned inverse-column-pass shape (0: default; 1: 1 pair per lane x 4
                           wavefronts, 2: 1 x 8) */
  int32_t cic_maxlog1;  /* tuned largest log2 L1 with the update fused (0: default) */
  int32_t tuned;        /* 0: not tuned, 1: timed at creation, 2: from the tuning cache */
  int64_t tune_batch;   /* batch size the choice was made for */
  double tune_us;       /* time of the chosen variant on tune_batch signals (microseconds) */
} slepian_plan_info;

typedef struct {
  int iterations;           /* refinement sweeps taken */
  double rel_residual;      /* max over the batch of ||By - (B^2+alpha I)x|| / ||By|| (Tikhonov) */
  double rel_residual_first;/* the same for the unrefined fast solution */
  int converged;            /* 1 if rel_residual <= tol */
} slepian_lsq_report;

/* Plan for length-N signals, half bandwidth W, tolerance eps, default options.
 * Setup (Section 1.3 "fast precomputation", Section 4.1): the spectrum of the
 * circulant embedding of B's first column, and the Slepian vectors with
 * eps < lambda < 1-eps, from bisection and inverse iteration on the
 * tridiagonal matrix that commutes with B (Slepian 1978) in FP64 on the GPU,
 * with lambda_l = s_l^T B s_l in FP64.  Synchronous.  *out receives a new
 * plan on success and is untouched on failure.
 * Errors: EINVAL (domain), EGAP, ENOMEM, EHIP, ENOCONV. */
int slepian_plan(int64_t N, double W, double eps, slepian_plan_t *out);

/* As slepian_plan with options (opts may be NULL for defaults). */
int slepian_plan_ex(int64_t N, double W, double eps, const slepian_plan_opts *opts,
                    slepian_plan_t *out);

/* Many plans at once (Section 4.1 setup for each): plan i for N[i], W[i],
 * eps[i] with options opts[i] (opts NULL: defaults for all; every plan on one
 * device).  The same plans as n calls of slepian_plan_ex, with the
 * eigensolves of all plans run together (one bisection, one inverse
 * iteration and one normalisation launch per memory batch), which keeps the
 * GPU busy where one plan's few hundred eigenvalues cannot.  Synchronous.
 * out: n handles, written only on success; on any error no plan is created
 * and the first failing status is returned (EINVAL, EGAP, ENOCONV, ENOMEM,
 * EHIP). */
int slepian_plan_batch(int n, const int64_t *N, const double *W, const double *eps, const slepian_plan_opts *opts,
                       slepian_plan_t *out);

/* Plan sizes and eigen-structure; info is host memory. */
int slepian_plan_info_get(slepian_plan_t plan, slepian_plan_info *info);

/* Eigenpairs held by the plan: the union of the transition sets it uses,
 * indices l = *l_first .. *l_first + *count - 1.  lam_host (host, may be
 * NULL) receives count FP64 eigenvalues; vecs (device, may be NULL) receives
 * the N x count FP64 unit-norm vectors, column-major with leading dimension
 * ldv >= N, each signed so that its first entry of magnitude >= 1e-3 of its
 * largest magnitude is positive.  cap is the capacity (in eigenpairs) of
 * lam_host/vecs; ENOMEM if smaller than count.  Synchronous. */
int slepian_plan_eigenpairs(slepian_plan_t plan, int64_t *l_first, int64_t *count,
                            double *lam_host, double *vecs, int64_t ldv, int64_t cap);

/* Write / read a plan (spectrum, vectors, eigenvalues, sizes) to / from a
 * file, so setup is not repeated.  load creates the plan on `device`
 * (-1: current). Errors: EIO, ENOMEM, EHIP. */
int slepian_plan_save(slepian_plan_t plan, const char *path);
int slepian_plan_load(const char *path, int device, slepian_plan_t *out);

/* Free a plan and its device buffers (NULL is a no-op). */
int slepian_plan_destroy(slepian_plan_t plan);

/* Workspace bytes needed by `op` on `batch` signals. */
int slepian_workspace_size(slepian_plan_t plan, int op, int64_t batch, size_t *bytes);

/* Fast projection onto span(S_K) (Corollary 2, Lemma 4; Section 1.3 "Fast
 * projections onto the range of S_K"):
 *     y = B x + U diag(d) U^T x,
 * U = the transition vectors (eps < lambda < 1-eps), d = 1 - lambda for
 * l < K and -lambda for l >= K, so ||y - S_K S_K^T x|| <= eps ||x|| plus
 * FP32 rounding.  B x uses length-L FFTs (L the smallest power of two >= 2N).
 * x: N x batch FP32 (ldx >= N); y: N x batch FP32 (ldy >= N); y may equal x
 * (in place) but must not otherwise overlap it.  batch == 0 is a no-op. */
int slepian_project(slepian_plan_t plan, const float *x, int64_t ldx, float *y, int64_t ldy,
                    int64_t batch, void *work, size_t work_bytes, void *stream);

/* slepian_project without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, result and precision as
 * slepian_project with work = NULL; its workspace is instead a fixed 160 MiB
 * device array inside the library (one per device, held until the process
 * ends).  A batch whose workspace exceeds it runs as consecutive sub-batches
 * of an even number of signals, the largest that fits, with the same
 * results.  The array is shared by every call on a device and keeps the last
 * call's contents: calls that overlap in time on one device (different
 * streams, different threads) race; serialise them.  Returns
 * SLEPIAN_ESCRATCH if even two signals do not fit (not reachable for
 * N <= 2^21), else as slepian_project.  No hipMalloc, hipFree or allocating
 * library call is made. */
int slepian_project_noalloc(slepian_plan_t plan, const float *x, int64_t ldx, float *y, int64_t ldy,
                            int64_t batch, void *stream);

/* As slepian_project with an explicit correction precision (enum
 * slepian_precision) instead of the plan's default. */
int slepian_project_ex(slepian_plan_t plan, int precision, const float *x, int64_t ldx,
                       float *y, int64_t ldy, int64_t batch, void *work, size_t work_bytes,
                       void *stream);

/* Multiband (modulated Slepian) dictionaries (Section 1.4, application i:
 * the Slepian basis modulated to several frequency bands and merged).  Band
 * centres freqs[i] (cycles/sample; 0 for the baseband band, otherwise
 * W <= f <= 1/2 - W; centres at least 2W apart, so the bands [f - W, f + W]
 * do not overlap); the dictionary of a real signal is {E_f S_K} over
 * f in {+-f_i}, E_f = diag(exp(2 pi i f n)).  Three calls:
 *   - slepian_project_bands_span (prepared band set): the orthogonal
 *     projection onto the dictionary's span;
 *   - slepian_project_bands (prepared band set) and slepian_project_multiband
 *     (no setup): the BAND SUM
 *         y = sum_i w_i Re(E_i P~ E_i^* x),
 *     w_i = 2 for f_i > 0 (the band pair +-f_i of a real signal), 1 for
 *     f_i = 0, P~ the plan's fast projection (Corollary 2).  The band sum is
 *     not a projection: the modulated subspaces are not orthogonal, and it
 *     differs from the projection onto their span by their overlap (0.3% to
 *     1.2% relative for white noise at N = 512..1024, W = 1/32, four bands).
 *     It is the operator the span projection iterates on.
 * slepian_project_multiband: band by band, in the plan's precision.  x, y:
 * N x batch FP32 real (y may equal x, no other overlap); 1 <= nbands <= 64;
 * EINVAL on bad bands.  Workspace: slepian_workspace_size(plan,
 * SLEPIAN_OP_MULTIBAND, nbands * batch). */
int slepian_project_multiband(slepian_plan_t plan, int nbands, const double *freqs, const float *x, int64_t ldx,
                              float *y, int64_t ldy, int64_t batch, void *work, size_t work_bytes, void *stream);

/* Prepared band set, computed with one FFT product instead of one per band.
 * For real x, Re(E_f B E_f^* x) is the Toeplitz product with the kernel
 * cos(2 pi f m) sin(2 pi W m)/(pi m), so the bands' B parts add up to one real
 * symmetric Toeplitz product, whose circulant spectrum (FP64 transform, stored
 * FP32) and a table of cos(2 pi f_i n), -sin(2 pi f_i n) (2 nbands x N FP32)
 * are built here; the correction parts form one correction of rank
 * 2 nbands r (r = the plan's transition count, at most 128, else ENOTSUP),
 * in the plan's precision (FP32, or BF16 hi/lo operands for MIXED and
 * BF16_RAW).  The band sum equals slepian_project_multiband's up to FP32
 * rounding.  The band rules and errors are slepian_project_multiband's; the
 * plan must outlive the band set.  Setup is synchronous. */
int slepian_bands_create(slepian_plan_t plan, int nbands, const double *freqs, slepian_bands_t *out);
int slepian_bands_destroy(slepian_bands_t bands);
/* Workspace bytes of slepian_project_bands on `batch` signals. */
int slepian_bands_workspace_size(slepian_bands_t bands, int64_t batch, size_t *bytes);
/* The band sum y = sum_i w_i Re(E_i P~ E_i^* x) for the prepared bands; x, y:
 * N x batch FP32 real (y may equal x, no other overlap); batch == 0 is a
 * no-op; ENOTSUP when the batch exceeds the launch limits of the correction. */
int slepian_project_bands(slepian_bands_t bands, const float *x, int64_t ldx, float *y, int64_t ldy,
                          int64_t batch, void *work, size_t work_bytes, void *stream);
/* Workspace bytes of slepian_project_bands_span on `batch` signals. */
int slepian_bands_span_workspace_size(slepian_bands_t bands, int64_t batch, size_t *bytes);
/* The orthogonal projection of each real signal onto the span of the band
 * set's modulated Slepian dictionary, by conjugate gradients on the band sum
 * A (above): A z = A x from z = 0, so the iterates stay in A's range, whose
 * solution is that projection when the bands' projections are exact.  Per
 * signal: a = rr / (p . Ap), z += a p, r -= a Ap, beta = rr_new / rr,
 * p = r + beta p, stopping once ||r|| <= tol ||A x|| (before the iteration
 * starts to resolve the eigenvalues of at most about eps that the fast
 * projections leave outside the span).  Vectors FP32, dot products and
 * scalars FP64 in a fixed order, A in the plan's precision.  Result within a
 * few eps ||x|| of the exact projection onto the span (the bound the tests
 * hold: 2 J eps, J the number of modulated bases).  tol = 0 selects
 * max(eps, 1e-6); else 1e-6 <= tol < 1/2.  1 <= max_iter <= 1000.  x, y:
 * N x batch FP32 (y may equal x, no other overlap).  iters (host, nullable,
 * batch entries) receives each signal's steps.  Synchronous (one small
 * device-to-host copy per step).  Returns SLEPIAN_ENOCONV, with y holding
 * the last iterate, if some signal has not met tol after max_iter steps. */
int slepian_project_bands_span(slepian_bands_t bands, const float *x, int64_t ldx, float *y, int64_t ldy,
                               int64_t batch, double tol, int max_iter, void *work, size_t work_bytes,
                               void *stream, int *iters);

/* Fast factorization S_K S_K^T ~= T1 T2^T (Section 1.3, "A fast
 * factorization", with Theorem 1):
 *     T1 = [F, L1, U diag(d)],   T2 = [F, L2, U],
 * F the partial DFT matrix of the 2NW' lowest length-N frequencies (2NW' =
 * kf, the odd integer nearest to 2NW; ties upward), L1 L2^* an approximation
 * of B - F F^* within eps of rank r1 (Theorem 1), and U diag(d) U^T the
 * plan's transition correction of Corollary 2.  ||S_K S_K^T - T1 T2^T|| <=
 * 2 eps.  For real signals F is used in its real form F_r (same F F^*):
 * columns 1/sqrt(N), sqrt(2/N) cos(2 pi k n / N), -sqrt(2/N) sin(2 pi k n / N)
 * for k = 1 .. (kf - 1)/2, in that interleaved order.  A compressed signal
 * holds kprime = kf + r1 + r FP32 numbers: [F_r^T x; L2^T x; U^T x].
 *
 * The two ways to get L1, L2 (enum slepian_factor_method):
 *  - SLEPIAN_FACTOR_THEOREM1 (default): the construction in the proof of
 *    Theorem 1 (Section 2).  B - F F^* splits into modulated copies of the
 *    Hilbert matrix, a remainder A1 and a matrix B0 (eq. (BA0), eq. (A0A1));
 *    the Hilbert matrix gets a CF-ADI factor with rH = ceil(log(8N-4)
 *    log(4 pi / delta_H) / pi^2) columns and elliptic-function shifts (Lemma 2
 *    and its proof in the appendix), A1 and B0 truncated power series of 2 rA
 *    and 2 rB - 1 terms, with delta_H = 4 pi eps / 15 and delta_A = delta_B =
 *    7 eps / 30.  r1 = 4 rH + 4 rA + 2 (2 rB - 1).  For real signals the
 *    complex L1, L2 (columns in conjugate pairs) are used in a real form with
 *    the same product.  The modulation D_B is diag(e^{j pi (W + W') n}).
 *    Setup (synchronous): the shifts and the series coefficients on the host,
 *    the N x r1 factors by one FP64 kernel (FP32 results).
 *  - SLEPIAN_FACTOR_EIG: L1 = V diag(mu), L2 = V, the eigenpairs of the
 *    symmetric Toeplitz matrix B - F F^* with |mu| > eps (the least rank for
 *    that error).  Setup (synchronous, FP64): subspace iteration on a random
 *    +-1 block with the FFT-applied B - F F^*, Householder QR and a
 *    Rayleigh-Ritz step (rocSOLVER), widening the block until the kept
 *    pairs have residuals of at most eps / 4 (checked with one more product)
 *    and six block power steps on the operator deflated by them (a fresh
 *    random block of 8 columns) find no eigenvalue above eps outside their
 *    span; ENOCONV if the block reaches its cap (1024) first.
 *
 * Requires N a power of two (the plan's FFT length is then exactly 2N) with
 * 256 <= N <= 2^20, else ENOTSUP.  The plan must outlive the factorization. */
typedef struct slepian_factor_s *slepian_factor_t;
enum slepian_factor_method {
  SLEPIAN_FACTOR_THEOREM1 = 0,
  SLEPIAN_FACTOR_EIG = 1
};
typedef struct {
  int64_t kf;         /* 2NW': rows of the F part of a compressed signal */
  int64_t r1;         /* columns of L1 and L2 */
  int64_t r;          /* columns of U (the plan's projection transition set) */
  int64_t kprime;     /* kf + r1 + r */
  int64_t subspace;   /* EIG: block size the setup converged with; THEOREM1: 0 */
  double mu_dropped;  /* EIG: largest |Ritz value| of B - F F^* left out (<= eps); THEOREM1: 0 */
  double ritz_residual; /* EIG: largest ||(B - F F^*) v - mu v|| of the kept pairs (<= eps / 4) */
  int32_t method;     /* enum slepian_factor_method */
  int32_t r_h, r_a, r_b; /* THEOREM1: rH, rA, rB of the construction; EIG: 0 */
  double deflated_norm; /* EIG: estimated largest |mu| outside the kept pairs' span (<= eps); THEOREM1: 0 */
} slepian_factor_info_t;
/* slepian_factor_create_ex with SLEPIAN_FACTOR_THEOREM1. */
int slepian_factor_create(slepian_plan_t plan, slepian_factor_t *out);
int slepian_factor_create_ex(slepian_plan_t plan, int method, slepian_factor_t *out);
int slepian_factor_destroy(slepian_factor_t f);
int slepian_factor_info(slepian_factor_t f, slepian_factor_info_t *info);
/* EIG: mu (r1 values, decreasing |mu|) to host memory of n >= r1 doubles;
 * THEOREM1: ENOTSUP (the construction has no eigenvalues). */
int slepian_factor_mu(slepian_factor_t f, double *mu, int64_t n);
/* Workspace bytes of compress or recover on `batch` signals. */
int slepian_factor_workspace_size(slepian_factor_t f, int64_t batch, size_t *bytes);
/* c = T2^T x.  x: N x batch FP32 (device, ldx >= N); c: kprime x batch FP32
 * (device, ldc >= kprime), no overlap with x.  F_r^T x runs through the
 * plan's FP32 FFT passes; L2^T x and U^T x as one product on the matrix cores
 * in the plan's precision (FP32, or BF16 hi/lo operands with FP32
 * accumulation).  batch == 0 is a no-op; batch <= 32 * 65535. */
int slepian_factor_compress(slepian_factor_t f, const float *x, int64_t ldx, float *c, int64_t ldc, int64_t batch,
                            void *work, size_t work_bytes, void *stream);
/* y = T1 c.  c: kprime x batch FP32 (ldc >= kprime); y: N x batch FP32
 * (ldy >= N), no overlap with c.  F_r c_F through the plan's FP32 inverse FFT
 * passes, then y += [L1 U] ([1 d] . c_rest) on the matrix cores in the
 * plan's precision (FP32, or BF16 hi/lo operands with FP32 accumulation),
 * fused into the inverse column pass where that pass takes the update. */
int slepian_factor_recover(slepian_factor_t f, const float *c, int64_t ldc, float *y, int64_t ldy, int64_t batch,
                           void *work, size_t work_bytes, void *stream);

/* Slepian coefficients c = S_K^T x (Section 1.3, "A fast factorization":
 * the K numbers that represent x), exact (dense) semantics.  The first call
 * computes all K Slepian vectors on the GPU and keeps them in the plan
 * (N*K*4 bytes, plus as many again for their BF16 hi/lo halves in plans of
 * MIXED or BF16_RAW precision); ENOTSUP if N*K*4 bytes exceed 16 GiB.  The
 * product runs on the library's own matrix-core GEMM: FP32 matrix
 * instructions for FP32 plans, otherwise three BF16 products of the hi/lo
 * halves (hi*hi + hi*lo + lo*hi) accumulated in FP32; partial sums over
 * the sample dimension are added in a fixed order, so results are
 * reproducible.  Vector signs follow the convention of
 * slepian_plan_eigenpairs.  c: K x batch FP32, ldc >= K, no overlap with x;
 * EHIP if a launch fails. */
int slepian_coeffs(slepian_plan_t plan, const float *x, int64_t ldx, float *c, int64_t ldc,
                   int64_t batch, void *work, size_t work_bytes, void *stream);

/* Least squares with the prolate matrix (Section 1.3):
 *   SLEPIAN_PINV:      x = B_K^+ y ~= B y + U diag(1/lambda - lambda | -lambda) U^T y
 *                      (Corollary 3, error <= 3 eps ||y||); single pass, tol and
 *                      max_iter ignored.  B y is the FP32 product; the
 *                      correction runs in FP64 (its weights 1/lambda, up to
 *                      1/eps, would amplify FP32 rounding of U^T y).  K is
 *                      the plan's (round(2NW) or the override of
 *                      slepian_plan_ex, e.g. #{lambda >= threshold}).
 *   SLEPIAN_TIKHONOV:  x ~= (B^2 + alpha I)^{-1} B y, starting from the fast
 *                      operator B y/(1+alpha) + U5 U5^T y (Corollary 4, error
 *                      <= eps ||y||; with max_iter = 0 the correction runs in
 *                      FP64, as its weights reach 1/(2 sqrt(alpha))), then
 *                      refined: with the FP64 residual
 *                      rho = B y - (B^2 + alpha I) x, x += M rho, where M is an
 *                      FP32 fast approximation of (B^2 + alpha I)^{-1}, until
 *                      max_s ||rho_s|| / ||B y_s|| <= tol or max_iter sweeps.
 *                      B x and B^2 x of the starting point come from FP64
 *                      products; each correction e then adds B e and B (B e)
 *                      from FP32 products (rounding near 1e-7 ||e||, far
 *                      below the tolerance), so a sweep costs two FP32
 *                      products and the fast operator M.  The residual so
 *                      tracked (reported in rep) lies within about 1e-13 of
 *                      ||B y|| of the one recomputed from scratch in FP64;
 *                      convergence requires it to be <= tol - 1e-12, so a
 *                      tol <= 1e-12 ends in ENOCONV after max_iter sweeps.
 *                      max_iter = 0 returns the fast operator's output.  alpha
 *                      must equal the plan's alpha (opts.alpha).
 * y: N x batch FP32; x: N x batch FP64 (FP64 so that the refined residual can
 * reach 1e-10).  rep (host, nullable) receives iterations and residuals; a
 * non-NULL rep or max_iter > 0 makes the call synchronous (the convergence
 * test reads norms on the host).  ENOCONV if tol is not reached. */
int slepian_lsq(slepian_plan_t plan, int mode, double alpha, const float *y, int64_t ldy,
                double *x, int64_t ldx, int64_t batch, double tol, int max_iter,
                void *work, size_t work_bytes, void *stream, slepian_lsq_report *rep);

/* FP64 product y = B x with the same FFT method (used for residuals). */
int slepian_apply_b64(slepian_plan_t plan, const double *x, int64_t ldx, double *y,
                      int64_t ldy, int64_t batch, void *work, size_t work_bytes, void *stream);

/* Groups: many independent plans (any mix of N, W, eps) projected together.
 * plans (host array of n plan handles) must outlive the group; batch (host)
 * gives each plan's signal count.  The group owns its workspace and a HIP
 * graph of the whole batch, built on the first slepian_group_project call and
 * re-launched as one graph while the pointer arrays stay the same.  Plans
 * are sorted into kernel classes (single-pass rows of 2^9..2^13 points with
 * or without the correction inside; three-pass rows of 2^13 points by L1),
 * one grouped launch per class and pass.  The first call tunes the launch
 * variants that have alternatives (signals per workgroup of the correction
 * partials; wavefronts per workgroup of each fused inverse column pass) by
 * timing them on the group's own data, or takes them from the tuning cache
 * of the first plan created with opts.tune_cache (an entry keyed by a hash of
 * every plan's N, W, eps, precision and batch), appending new choices. */
int slepian_group_create(const slepian_plan_t *plans, int n, const int64_t *batch,
                         slepian_group_t *out);
typedef struct {
  int32_t plans, grouped, other;  /* plans; in the graph's grouped launches; run plan by plan */
  int32_t tuned;                  /* 0: not yet, 1: timed, 2: from the tuning cache */
  int32_t partial_variant;        /* correction partials: 0 64, 1 32 signals per workgroup */
  int32_t cic_variant[5];         /* fused inverse column pass at L1 = 2..32: 0 8, 1 4 wavefronts */
} slepian_group_info_t;
int slepian_group_info(slepian_group_t group, slepian_group_info_t *info);

/* x, y: host arrays of n device pointers; plan i reads x[i] (N_i x batch_i,
 * ld N_i) and writes y[i] (same shape).  Asynchronous on `stream`. */
int slepian_group_project(slepian_group_t group, const float *const *x, float *const *y,
                          void *stream);

int slepian_group_destroy(slepian_group_t group);

/* Kernel tracing (profiling).  While enabled (process-wide, off by default),
 * every hot-path kernel launch of the library is bracketed by two HIP events
 * recorded on the launch's own stream, so the elapsed time between them is
 * that kernel's device duration.  slepian_trace_read synchronises on the
 * recorded events and returns per-kernel totals (name, launches, total/min/max
 * milliseconds) into stats (host, cap entries); *count receives the number of
 * distinct kernels (may exceed cap).  reset != 0 clears the records.  Tracing
 * adds two event records per launch; do not enable it while a stream is being
 * captured into a graph. */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms, min_ms, max_ms;
} slepian_kernel_stat;

int slepian_trace_enable(int on);
int slepian_trace_read(slepian_kernel_stat *stats, int cap, int *count, int reset);

/* Static description of a status code. */
const char *slepian_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* SLEPIAN_H_ */

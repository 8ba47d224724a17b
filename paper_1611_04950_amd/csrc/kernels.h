// Host-side launchers of the HIP kernels (internal to libslepian).
#pragma once

#include "common.h"

namespace slp {

// ---- FFT product (fft.hip, fft2.hip) ----
// Geometry for transform length 2^logL with at most 2^logE points per
// workgroup; register-stage kernels where a row shape and column length fit.
FftGeom make_geom(int logL, int logE, bool allow_v2);
FftGeom generic_twin(const FftGeom &g);

template <typename R>
hipError_t build_row_tables(const FftGeom &g, cpx<R> *rt1, cpx<R> *rt2, hipStream_t st);
template <typename R>
hipError_t build_col_table(const FftGeom &g, cpx<R> *tc, hipStream_t st);

// U columns of the fused inverse column pass's tile (r padded to its matrix step:
// 16 for mode 0, 32 for mode 1)
int colinv_corr_rp(int r, int mode);
// whether the inverse column pass carries the correction update (L1 = 2^log1 <= 16,
// or <= 32 with the tuning override; output leading dimension ldy, b signals, rank r
// within its 32-bit offsets), and whether a plan of that L1 keeps the tiles it reads
bool colinv_corr_ok(const FftGeom &g, int64_t ldy, int64_t b, int r);
bool colinv_corr_tiled(const FftGeom &g);
// U's rows laid out for the fused inverse column pass (mode 0: FP32; mode 1: BF16 hi
// and lo planes); bytes, and the layout kernel (U: N x r, leading dimension ldu)
size_t corr_tile_bytes(int log1, int log2, int r, int mode);
hipError_t build_corr_tile(const float *U, int64_t ldu, int N, int r, int log1, int log2, int mode, void *out,
                           hipStream_t st);

// Pass A fused with the correction's coefficients C = U^T x (L1 = 16 or 32,
// rank 1..32): Z as pass A writes it, and one partial of C per column block
// of 16 columns (colfwd_corr_chunks of them, layout of the chunk sum) into
// part; ft from build_fwd_tile for the same geometry, rank and mode (0: FP32,
// 1: BF16 hi/lo).  One slice: all (b + 1) / 2 pairs in Z.
bool colfwd_corr_ok(const FftGeom &g, int r);
int colfwd_corr_chunks(const FftGeom &g);
size_t fwd_tile_bytes(const FftGeom &g, int r);
hipError_t build_fwd_tile(const float *U, int64_t ldu, int N, int r, const FftGeom &g, int mode, void *out,
                          hipStream_t st);
hipError_t colfwd_corr(const float *x, int64_t ldx, int64_t N, int64_t b, const FftGeom &g,
                       const FftTables<float> &tb, cpx<float> *Z, const void *ft, int r, int mode, float *part,
                       hipStream_t st);
// The rest of the product after colfwd_corr: rows (carrying the chunk sum of
// the coefficients into rs->dC when rs is set), then the inverse column pass
// (with the update when corr.dC is set).
hipError_t conv_rows_inv(float *y, int64_t ldy, int64_t N, int64_t b, const FftGeom &g, const FftTables<float> &tb,
                         float beta, float gamma, const Corr<float> &corr, cpx<float> *Z, const RowSum *rs,
                         hipStream_t st);

// ---- grouped launches over many plans (fft2.hip, corr_mfma.hip) ----
// Workgroups each plan contributes to a grouped launch.
int64_t group_blocks_single(const GroupPlan &P);
int64_t group_blocks_colfwd(const GroupPlan &P);
int64_t group_blocks_row(const GroupPlan &P);
int64_t group_blocks_colinv(const GroupPlan &P, int cw);  // cw: wavefronts per workgroup (4 or 8)
int64_t group_blocks_partial(const GroupPlan &P, int nb);  // nb: 32-signal blocks per wavefront (1 or 2)
int64_t group_blocks_reduce(const GroupPlan &P);
// single-pass product (with the fused FP32 correction when `corr`), all plans of row length 2^log2
hipError_t group_single(int log2, bool corr, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st);
// plain inverse column pass (the correction update follows separately)
hipError_t group_colinv(int log1, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st);
// y += U dC on the matrix cores for every plan of the span
int64_t group_blocks_apply(const GroupPlan &P);
hipError_t group_corr_apply(bool vec, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st);
// three-pass passes; all plans of the span share L1 = 2^log1 (columns) or L2 = 2^log2 (rows)
hipError_t group_colfwd(int log1, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st);
hipError_t group_row(int log2, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st);
// one: plans whose single-plan pass takes the single-step contraction (L1 =
// 32, rank <= 32; colinv_corr_one)
hipError_t group_colinv_corr(int log1, int mode, int cw, bool one, const GroupPlan *gp, const GroupSpan &sp,
                             hipStream_t st);
bool colinv_corr_one(int log1, int rp);
int64_t group_blocks_colfwd_corr(const GroupPlan &P);
hipError_t group_colfwd_corr(int log1, int mode, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st);
// C = U^T x partials and dC = d (.) C for every plan of the span
hipError_t group_corr_partial(int mode, int nb, bool vec, const GroupPlan *gp, const GroupSpan &sp,
                              hipStream_t st);
hipError_t group_corr_reduce(const GroupPlan *gp, const GroupSpan &sp, hipStream_t st);

template <typename R>
hipError_t conv_apply_v2(const R *x, int64_t ldx, R *y, int64_t ldy, int64_t N, int64_t b, const FftGeom &g,
                         const FftTables<R> &tb, R beta, R gamma, const Corr<R> &corr, cpx<R> *Z, int64_t slice_pairs,
                         hipStream_t st);

template <typename R>
hipError_t build_tables(const FftGeom &g, cpx<R> *tw_sub, cpx<R> *tw_lo, cpx<R> *tw_hi, hipStream_t st);

hipError_t sinc_embed(double *c, int64_t L, int64_t N, double W, hipStream_t st);

hipError_t fft_forward_real64(const double *c, const FftGeom &g, const FftTables<double> &tb,
                              cpx<double> *spec, hipStream_t st);

template <typename R>
hipError_t spectrum_relayout(const cpx<double> *src, const FftGeom &gs, R *dst, const FftGeom &gd,
                             hipStream_t st);

size_t conv_workspace_pairs(const FftGeom &g, int64_t pairs, size_t elem_bytes, size_t budget);

template <typename R>
hipError_t conv_apply(const R *x, int64_t ldx, R *y, int64_t ldy, int64_t N, int64_t b, const FftGeom &g,
                      const FftTables<R> &tb, R beta, R gamma, const Corr<R> &corr, cpx<R> *Z,
                      int64_t slice_pairs, hipStream_t st);

// ---- Tridiagonal eigensolver and Rayleigh quotients (eig.hip) ----
hipError_t tridiag_build(double *a, double *e2, int64_t N, double W, hipStream_t st);

// Eigenvalues theta_t (ascending order index t = t0 .. t0+count-1) of the
// tridiagonal matrix by multisection on Sturm counts.
hipError_t tridiag_bisect(const double *a, const double *e2, int64_t N, double gl, double gu, double pivmin,
                          int64_t t0, int64_t count, double *theta, hipStream_t st);

// Inverse iteration for `count` eigenvalues; writes unit-norm, sign-fixed
// vectors to V (N x count, column-major, ld N), column order reversed
// (column count-1-j holds theta[j]) so columns run in descending theta.
// `scratch` must hold inviter_scratch_bytes(N, count) bytes.
size_t inviter_scratch_bytes(int64_t N, int64_t count);
hipError_t tridiag_inviter(const double *a, const double *off, int64_t N, const double *theta, int64_t count,
                           double *V, void *scratch, int iters, hipStream_t st);

// lam[j] = v_j^T (B v_j), res[j] = ||B v_j - lam_j v_j|| for unit v_j.
// Many plans' eigensolves in three launches (bisection, inverse iteration,
// normalisation), each job solving `count` eigenvalues of its tridiagonal
// matrix from ascending index t0 into theta and the vectors into V (N x count,
// the same order as tridiag_inviter), with inviter_scratch_bytes(N, count)
// bytes of scratch.  Synchronous.
struct EigJob {
  const double *a, *e2, *off;
  int64_t N, t0, count;
  double gl, gu, pivmin;
  double *theta, *V;
  void *scratch;
};
hipError_t eig_solve_many(const EigJob *jobs, int m, int iters, hipStream_t st);

// ---- Multiband dictionaries (multiband.hip) ----
constexpr int kMaxBands = 64;
struct BandSet {  // band centres (cycles/sample), passed by value to the kernels
  int J = 0;
  double f[kMaxBands];
};
// z: 2 J b signals (leading dimension ldz): the real and imaginary parts of
// E_{f_i}^* x_s at 2 (i b + s) and 2 (i b + s) + 1
hipError_t band_demod(const float *x, int64_t ldx, int64_t N, int64_t b, const BandSet &bs, float *z, int64_t ldz,
                      hipStream_t st);
// y_s = sum_i w_i Re(E_{f_i} (p_{2(ib+s)} + i p_{2(ib+s)+1})), w_i = 2 (f_i > 0) or 1 (f_i = 0)
hipError_t band_remod(const float *p, int64_t ldp, int64_t N, int64_t b, const BandSet &bs, float *y, int64_t ldy,
                      hipStream_t st);
// Prepared band sets: circulant embedding (length L, FP64) of the band-sum kernel
// b(m) sum_i w_i cos(2 pi f_i m), and the modulation table M[(2 i + c) ldm + n]
// (c = 0: cos(2 pi f_i n), c = 1: -sin(2 pi f_i n); zero for N <= n < ldm, ldm a
// multiple of 64) with band_table_rows(J) = 2 J + 1 rows, the last one zero
hipError_t band_embed(double *c, int64_t L, int64_t N, double W, const BandSet &bs, hipStream_t st);
int64_t band_table_rows(int J);
int64_t mb_ldm(int64_t N);  // leading dimension of the table and of U's [j][n] planes
hipError_t band_table(float *M, int64_t ldm, int64_t N, const BandSet &bs, hipStream_t st);
// The modulated correction of rank 2 J r: coefficients dC' from x (before the
// product, so that y may alias x), then y += the update.  mode 0 FP32, 1 BF16 hi/lo.
constexpr int kMbMaxRank = 128;
struct MbShape {
  int ncmb = 0, logG = 0, nsg = 0, nbw = 0, nw = 0, ncg = 0, nz = 0, rpad = 0, jp = 0, steps = 0, chunks = 0;
  int tiles = 0, cu = 0;  // apply: 16-sample tiles per wavefront, modulations per iteration
  int ss = 0, lds_bytes = 0;  // coefficients: samples per LDS stage, dynamic LDS bytes
};
struct MbWs {
  float *part = nullptr, *D = nullptr;
  __bf16 *H = nullptr, *Lo = nullptr;
};
// U's columns for the modulated correction (the plan's proj set), laid out by
// mb_ulayout once per plan and matrix mode: a copy blocked by 8 samples,
// [(n / 8) rpad + j] 8 + n % 8 with rpad = 32 ceil(r / 32) rows and n < ldm (BF16
// hi/lo planes Uh, Ul for mode 1, U32b in FP32 for mode 0), and U^T planes
// [n][rpad] (Th, Tl in BF16 for mode 1, T32 in FP32 for mode 0).  The table's
// blocking is the same: [(n / 8) (2J + 1) + row] 8 + n % 8.
struct MbU {
  const __bf16 *Uh = nullptr, *Ul = nullptr, *Th = nullptr, *Tl = nullptr;
  const float *U32b = nullptr, *T32 = nullptr;
};
hipError_t mb_ulayout(int mode, const float *U, int64_t ldu, int64_t N, int r, int64_t ldm, __bf16 *Uh, __bf16 *Ul,
                      float *U32b, __bf16 *Th, __bf16 *Tl, float *T32, hipStream_t st);
MbShape mb_shape(int64_t N, int64_t b, int r, int J);
bool mb_ok(const MbShape &sh, int64_t N, int64_t b, int r);
size_t mb_workspace_bytes(const MbShape &sh, int64_t b);
MbWs mb_carve(const MbShape &sh, int64_t b, void *ws);
hipError_t mb_coeffs(int mode, const float *x, int64_t ldx, int64_t N, int64_t b, const MbU &u, int r,
                     const float *d, const float *M, int64_t ldm, const BandSet &bs, const MbShape &sh, const MbWs &w,
                     hipStream_t st);
hipError_t mb_apply(int mode, float *y, int64_t ldy, int64_t N, int64_t b, const MbU &u, int r, const float *M,
                    int64_t ldm, const MbShape &sh, const MbWs &w, hipStream_t st);

hipError_t rayleigh(const double *V, const double *BV, int64_t N, int64_t count, double *lam, double *res,
                    hipStream_t st);

// ---- Low-rank correction of the pseudoinverse in FP64 (corr.hip) ----
int corr_rpad(int r);  // r rounded up to the 32-column matrix tiles
// x += U diag(d) U^T y for the FP32 signals y (FP64 products and sums, x FP64);
// U: N x r FP64, leading dimension ldu; part and dC: corr64_workspace_doubles.
hipError_t corr64(const float *y, int64_t ldy, double *x, int64_t ldx, int64_t N, int64_t b, const double *U,
                  int64_t ldu, int r, const double *d, double *part, double *dC, hipStream_t st);
size_t corr64_workspace_doubles(int64_t N, int64_t b, int r);

// ---- Small elementwise helpers (eig.hip) ----
hipError_t cast_f64_to_f32(const double *src, int64_t ld_src, float *dst, int64_t ld_dst, int64_t rows,
                           int64_t cols, hipStream_t st);
hipError_t cast_f32_to_f64(const float *src, int64_t ld_src, double *dst, int64_t ld_dst, int64_t rows,
                           int64_t cols, hipStream_t st);

// ---- Low-rank correction on the matrix cores (corr_mfma.hip) ----
// mode: 0 FP32, 1 BF16 hi/lo (three products), 2 BF16 only.
int corr_nchunks(int64_t N, int64_t b, int r);
hipError_t corr_partial_mfma(int mode, const float *x, int64_t ldx, int64_t N, int64_t b, const float *U,
                             int64_t ldu, int r, float *part, hipStream_t st);
hipError_t corr_reduce_mfma(const float *part, int64_t N, int64_t b, int r, const float *d, float *dC,
                            hipStream_t st);
// c[s * ldc + j] = sum over chunks (no weights)
hipError_t corr_sum_mfma(const float *part, int64_t N, int64_t b, int r, float *c, int64_t ldc, hipStream_t st);
hipError_t corr_apply_mfma(float *y, int64_t ldy, int64_t N, int64_t b, const float *U, int64_t ldu, int r,
                           const float *dC, hipStream_t st);

// ---- Slepian coefficients as a library GEMM (gemm.hip) ----
// dst (rows x cols, ldd) = src (lds), FP32
hipError_t copy_f32(const float *src, int64_t lds, float *dst, int64_t ldd, int64_t rows, int64_t cols,
                    hipStream_t st);

// ---- Slepian coefficients c = S_K^T x on the matrix cores (coeffs.hip) ----
// Operand images: columns in 32-sample steps of one 128-byte line each (mode
// 0: FP32 columns with leading dimension 32 coeffs_steps(N); mode 1: BF16
// hi/lo pieces, step-major), zero past N.
int64_t coeffs_steps(int64_t N);
size_t coeffs_image_bytes(int64_t N, int64_t ncols);
hipError_t coeffs_image(int mode, const float *src, int64_t lds, int64_t N, int64_t ncols, void *dst,
                        hipStream_t st);
// Reduction splits of one GEMM and the floats of its partial tiles.
int coeffs_splits(int mode, int64_t N, int64_t K, int64_t b);
size_t coeffs_part_floats(int64_t N, int64_t K, int64_t b);
// c (K x b, ldc) = S^T X from the images of S (K columns) and X (b <= 65535
// columns); part holds coeffs_part_floats(N, K, b) floats.
hipError_t coeffs_gemm(int mode, const void *Simg, const void *Ximg, int64_t N, int64_t K, int64_t b, float *part,
                       float *c, int64_t ldc, hipStream_t st);

// ---- Conjugate gradients on a multiband band-sum operator (mbcg.hip) ----
constexpr int kCgChunk = 8192;  // samples per chunk of the fixed-order FP64 dot products
struct CgState {
  double rr, nb2, a, beta;  // ||r||^2, ||A x||^2, step, direction weight
  int iters, active, upd;   // steps taken; still iterating; direction updated in the last step
  int pad;
};
int cg_nchunks(int64_t N);
hipError_t cg_dot(const float *u, int64_t ldu, const float *v, int64_t ldv, int64_t N, int64_t b, double *part,
                  hipStream_t st);
hipError_t cg_init(const double *part, int64_t N, int64_t b, double tol, CgState *state, hipStream_t st);
hipError_t cg_alpha(const double *part, int64_t N, int64_t b, CgState *state, hipStream_t st);
hipError_t cg_update(float *z, int64_t ldz, float *r, const float *p, const float *ap, int64_t ldw, int64_t N,
                     int64_t b, const CgState *state, double *part, hipStream_t st);
hipError_t cg_beta(const double *part, int64_t N, int64_t b, double tol, CgState *state, hipStream_t st);
hipError_t cg_direction(float *p, const float *r, int64_t ldw, int64_t N, int64_t b, const CgState *state,
                        hipStream_t st);
hipError_t fill_zero_rows(float *y, int64_t ldy, int64_t N, int64_t b, hipStream_t st);
hipError_t copy_rows(const float *src, int64_t lds, float *dst, int64_t ldd, int64_t N, int64_t b, hipStream_t st);

// ---- Fast factorization T1 T2^T (fft2.hip, factor.hip) ----
// Length-N DFT bins |k| <= M = (kf - 1)/2 of signal pairs through the FP32
// product's geometry g (L = 2N): forward from x into Zb (kf bins per pair,
// slot M + k), and inverse from Zb into y (rows n < N), with y += U dC fused
// into the inverse column pass when corr.dC is set (three-pass geometries the
// fused pass handles; corr.ut from build_corr_tile).  dft_bins_ok: whether g
// supports them (register-stage row shape, L = 2N).
bool dft_bins_ok(const FftGeom &g, int64_t N);
hipError_t dft_bins_fwd(const float *x, int64_t ldx, int64_t N, int64_t b, const FftGeom &g,
                        const FftTables<float> &tb, cpx<float> *Z, int64_t slice_pairs, cpx<float> *Zb, int kf,
                        hipStream_t st);
hipError_t dft_bins_inv(const cpx<float> *Zb, int kf, float *y, int64_t ldy, int64_t N, int64_t b,
                        const FftGeom &g, const FftTables<float> &tb, cpx<float> *Z, int64_t slice_pairs,
                        const Corr<float> &corr, hipStream_t st);
// first column of B - F F^* embedded in a length-L circulant (FP64)
hipError_t diff_embed(double *c, int64_t L, int64_t N, double W, int kf, hipStream_t st);
// Rows of Theorem 1's real factor: prm = [shifts (rH) | C_A (2rA x 2rA) | C_B
// ((2rB-1) x (2rB-1))], row-major; L2 (compression) and L1 (recovery) get
// 2 (2 rH + 2 rA + 2 rB - 1) columns each, leading dimension ld.
hipError_t theorem1_rows(int64_t N, int kf, double W, int rH, int rA, int rB, const double *prm, float *L2,
                         float *L1, int64_t ld, hipStream_t st);
// N x p block of +-1 (FP64, leading dimension ld) from a counter-based generator
hipError_t rademacher(double *O, int64_t ld, int64_t N, int64_t p, uint64_t seed, hipStream_t st);
// sign convention of each column: first entry of magnitude >= 1e-3 max positive
hipError_t sign_fix_cols(double *V, int64_t ld, int64_t N, int64_t cols, hipStream_t st);
// R[:, j] -= mu[j] V[:, j] (FP64, N x r, leading dimension ld; mu on the device)
hipError_t ritz_residual(double *R, const double *V, const double *mu, int64_t ld, int64_t N, int64_t r,
                         hipStream_t st);
// pair bins -> the real coefficients F_r^T x (rows 0 .. kf-1 of c, leading dimension ldc)
hipError_t bins_unpack(const cpx<float> *Zb, int kf, int64_t N, int64_t b, float *c, int64_t ldc, hipStream_t st);
// recovery's reads of c: the real coefficients -> pair bins (Zb), and
// dC[j b + s] = w[j] c[kf + j + s ldc] (j < r)
hipError_t pack_scale(const float *c, int64_t ldc, int kf, int64_t N, int64_t b, cpx<float> *Zb, int r,
                      const float *w, float *dC, hipStream_t st);

// ---- Least-squares refinement helpers (lsq.hip) ----
// rho = By - u - alpha x formed in FP64 (N x b with leading dimension N except
// x: ldx), written to rho32 as FP32, with the column norms of the FP64 values
// (the same sums as col_norms; part: b * kNormParts doubles)
hipError_t lsq_residual_norms(const double *By, const double *u, const double *x, int64_t ldx, double alpha,
                              float *rho32, int64_t N, int64_t b, double *norms, double *part, hipStream_t st);
// norms[s] = ||v_s||_2 (FP64, fixed summation order); part: b * kNormParts doubles of scratch
constexpr int kNormParts = 256;
hipError_t col_norms(const double *v, int64_t ldv, int64_t N, int64_t b, double *norms, double *part,
                     hipStream_t st);
// x (FP64, ldx) += e (FP32, lde)
hipError_t add_f32_to_f64(const float *e, int64_t lde, double *x, int64_t ldx, int64_t N, int64_t b, hipStream_t st);

}  // namespace slp

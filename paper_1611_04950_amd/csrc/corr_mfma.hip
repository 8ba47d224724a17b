// Low-rank correction on the matrix cores (Corollaries 2-4, Lemmas 4-6):
//     C = U^T X  (r x N by N x b),   dC = d (.) C,   Y += U dC.
//
// The product C = U^T X is split over chunks of samples; each wavefront owns
// one 32-column block of U, a block of 32*NB signals and one chunk, and keeps
// NB 32 x 32 FP32 accumulators.  Operands are loaded straight from HBM in the
// matrix-core register layout: lane (i, kb) = (lane % 32, lane / 32) holds the
// eight consecutive samples k0 + 8 kb + e of U's column i and of signal i, so
// no LDS staging is needed.  Three arithmetic modes:
//   FP32       v_mfma_f32_32x32x2_f32, one instruction per sample pair;
//   MIXED      BF16 hi/lo split of both operands, three v_mfma_f32_32x32x16_bf16
//              per 16 samples (hi*hi + hi*lo + lo*hi), FP32 accumulation;
//   BF16_RAW   the hi*hi term only (for error studies).
// Chunk partials are summed in a fixed order (deterministic).
//
// The update Y += U dC loads a 32-sample x 32*NB-signal tile of Y into the
// accumulators (output layout: row 8 (v/4) + 4 (lane/32) + v % 4, column
// lane % 32), adds U dC with FP32 matrix instructions over j, and stores it.
#include "common.h"
#include "corr_sum.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum { kModeF32 = 0, kModeBF16x3 = 1, kModeBF16 = 2 };

__device__ __forceinline__ void split_bf16(const float (&v)[8], bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)v[e];
    hi[e] = h;
    lo[e] = (__bf16)(v[e] - (float)h);
  }
}

// One workgroup = 4 wavefronts on 4 consecutive chunks of KS*16 samples each;
// every wavefront issues all of its loads before its first matrix instruction,
// and the four accumulators are summed through LDS in a fixed order, so one
// partial per workgroup reaches memory.  With VEC (16-byte aligned leading
// dimensions and base pointers, checked by the caller) full chunks use
// branch-free float4 loads: lanes past the last signal or U column read a
// clamped valid address and are zeroed by a select, so all loads stay in
// flight together.  The one chunk that crosses N takes the checked path.
template <int MODE, int NB, int KS, bool VEC>
__device__ __forceinline__ void corr_partial_body(const float *__restrict__ X, int64_t ldx, int N, int b,
                                                  const float *__restrict__ U, int64_t ldu, int r,
                                                  float *__restrict__ part, int rpad, int bx, int by, int bz) {
  __shared__ float red[3][NB][16][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 31, kb = lane >> 5;
  const int s_base = by * 32 * NB;
  const int j = bz * 32 + i;
  const bool jv = j < r;
  constexpr int KC = KS * 16;
  const int k_begin = (bx * 4 + wave) * KC;
  const int k_end = min(N, k_begin + KC);
  const float *Uj = U + (int64_t)(jv ? j : r - 1) * ldu;
  float ua[KS][8];
  float xb[KS][NB][8];
  if (VEC && k_begin + KC <= N) {
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int kk = k_begin + 16 * q + 8 * kb;
      const float4 a0 = *reinterpret_cast<const float4 *>(Uj + kk);
      const float4 a1 = *reinterpret_cast<const float4 *>(Uj + kk + 4);
      ua[q][0] = a0.x; ua[q][1] = a0.y; ua[q][2] = a0.z; ua[q][3] = a0.w;
      ua[q][4] = a1.x; ua[q][5] = a1.y; ua[q][6] = a1.z; ua[q][7] = a1.w;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int s = s_base + nb * 32 + i;
        const float *xp = X + (int64_t)(s < b ? s : b - 1) * ldx + kk;
        const float4 c0 = *reinterpret_cast<const float4 *>(xp);
        const float4 c1 = *reinterpret_cast<const float4 *>(xp + 4);
        xb[q][nb][0] = c0.x; xb[q][nb][1] = c0.y; xb[q][nb][2] = c0.z; xb[q][nb][3] = c0.w;
        xb[q][nb][4] = c1.x; xb[q][nb][5] = c1.y; xb[q][nb][6] = c1.z; xb[q][nb][7] = c1.w;
      }
    }
#pragma unroll
    for (int q = 0; q < KS; ++q) {
#pragma unroll
      for (int e = 0; e < 8; ++e) ua[q][e] = jv ? ua[q][e] : 0.f;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bool v = s_base + nb * 32 + i < b;
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[q][nb][e] = v ? xb[q][nb][e] : 0.f;
      }
    }
  } else if (k_begin + KC <= N) {
    // full chunk, rows not 16-byte aligned: unguarded dword loads from
    // clamped rows, invalid lanes zeroed afterwards
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int kk = k_begin + 16 * q + 8 * kb;
#pragma unroll
      for (int e = 0; e < 8; ++e) ua[q][e] = Uj[kk + e];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int s = s_base + nb * 32 + i;
        const float *xp = X + (int64_t)(s < b ? s : b - 1) * ldx + kk;
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[q][nb][e] = xp[e];
      }
    }
#pragma unroll
    for (int q = 0; q < KS; ++q) {
#pragma unroll
      for (int e = 0; e < 8; ++e) ua[q][e] = jv ? ua[q][e] : 0.f;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bool v = s_base + nb * 32 + i < b;
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[q][nb][e] = v ? xb[q][nb][e] : 0.f;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int kk = k_begin + 16 * q + 8 * kb;
#pragma unroll
      for (int e = 0; e < 8; ++e) ua[q][e] = (jv && kk + e < k_end) ? Uj[kk + e] : 0.f;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int s = s_base + nb * 32 + i;
        const float *xp = X + (int64_t)(s < b ? s : 0) * ldx;
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[q][nb][e] = (s < b && kk + e < k_end) ? xp[kk + e] : 0.f;
      }
    }
  }
  f32x16 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[nb][v] = 0.f;
#pragma unroll
  for (int q = 0; q < KS; ++q) {
    if constexpr (MODE == kModeF32) {
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ua[q][e], xb[q][nb][e], acc[nb], 0, 0, 0);
    } else {
      bf16x8 ahi, alo;
      split_bf16(ua[q], ahi, alo);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        bf16x8 bhi, blo;
        split_bf16(xb[q][nb], bhi, blo);
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi, acc[nb], 0, 0, 0);
        if constexpr (MODE == kModeBF16x3) {
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo, acc[nb], 0, 0, 0);
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi, acc[nb], 0, 0, 0);
        }
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) red[wave - 1][nb][v][lane] = acc[nb][v];
  }
  __syncthreads();
  if (wave != 0) return;
  // D[row][col]: row = U column, col = signal
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int s = s_base + nb * 32 + i;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float t = (acc[nb][v] + red[0][nb][v][lane]) + (red[1][nb][v][lane] + red[2][nb][v][lane]);
      const int jj = bz * 32 + 8 * (v >> 2) + 4 * kb + (v & 3);
      if (jj < r && s < b) part[((int64_t)bx * rpad + jj) * b + s] = t;
    }
  }
}

// Workgroup (bx, by) of an nx x ny grid, dealt so that the ny workgroups of
// one bx (which share U's rows for those samples) run on one XCD: the
// dispatcher hands consecutive workgroups to the eight XCDs in turn, so the
// k-th workgroup of XCD x takes bx = 8 (k / ny) + x, by = k % ny.  Grids with
// nx not a multiple of 8 keep the plain order.
struct Blk2 {
  int bx, by;
};
__device__ __forceinline__ Blk2 xcd_blocks() {
  const int nx = gridDim.x, ny = gridDim.y;
  if (nx & 7) return Blk2{(int)blockIdx.x, (int)blockIdx.y};
  const int64_t l = (int64_t)blockIdx.x + (int64_t)nx * blockIdx.y;
  const int x = (int)(l & 7);
  const int64_t k = l >> 3;
  return Blk2{(int)(8 * (k / ny) + x), (int)(k % ny)};
}

template <int MODE, int NB, int KS, bool VEC>
__global__ __launch_bounds__(256) void k_corr_partial_mfma(const float *__restrict__ X, int64_t ldx, int N, int b,
                                                           const float *__restrict__ U, int64_t ldu, int r,
                                                           float *__restrict__ part, int rpad) {
  const Blk2 w = xcd_blocks();
  corr_partial_body<MODE, NB, KS, VEC>(X, ldx, N, b, U, ldu, r, part, rpad, w.bx, w.by, blockIdx.z);
}

// The same partials for r > 32 in one pass over x: each workgroup loads its
// chunk of x once (and, in the BF16 modes, splits it into hi/lo halves once)
// and then runs the nz = ceil(r / 32) column tiles of U in turn, each with
// the same matrix instructions, fixed-order wavefront sum through LDS and
// partial layout as corr_partial_body.
template <int MODE, int NB, int KS, bool VEC>
__global__ __launch_bounds__(256) void k_corr_partial_tiles(const float *__restrict__ X, int64_t ldx, int N, int b,
                                                            const float *__restrict__ U, int64_t ldu, int r,
                                                            float *__restrict__ part, int rpad, int nz) {
  __shared__ float red[3][NB][16][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 31, kb = lane >> 5;
  const int bx = blockIdx.x, by = blockIdx.y;
  const int s_base = by * 32 * NB;
  constexpr int KC = KS * 16;
  const int k_begin = (bx * 4 + wave) * KC;
  const int k_end = min(N, k_begin + KC);
  const bool full = k_begin + KC <= N;
  float xb[KS][NB][8];
#pragma unroll
  for (int q = 0; q < KS; ++q) {
    const int kk = k_begin + 16 * q + 8 * kb;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int s = s_base + nb * 32 + i;
      const bool v = s < b;
      const float *xp = X + (int64_t)(v ? s : b - 1) * ldx;
      if (VEC && full) {
        const float4 c0 = *reinterpret_cast<const float4 *>(xp + kk);
        const float4 c1 = *reinterpret_cast<const float4 *>(xp + kk + 4);
        xb[q][nb][0] = c0.x; xb[q][nb][1] = c0.y; xb[q][nb][2] = c0.z; xb[q][nb][3] = c0.w;
        xb[q][nb][4] = c1.x; xb[q][nb][5] = c1.y; xb[q][nb][6] = c1.z; xb[q][nb][7] = c1.w;
      } else if (full) {
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[q][nb][e] = xp[kk + e];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[q][nb][e] = kk + e < k_end ? xp[kk + e] : 0.f;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) xb[q][nb][e] = v ? xb[q][nb][e] : 0.f;
    }
  }
  bf16x8 xh[KS][NB], xl[KS][NB];
  if constexpr (MODE != kModeF32) {
#pragma unroll
    for (int q = 0; q < KS; ++q)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) split_bf16(xb[q][nb], xh[q][nb], xl[q][nb]);
  }
  for (int bz = 0; bz < nz; ++bz) {
    const int j = bz * 32 + i;
    const bool jv = j < r;
    const float *Uj = U + (int64_t)(jv ? j : r - 1) * ldu;
    float ua[KS][8];
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int kk = k_begin + 16 * q + 8 * kb;
      if (VEC && full) {
        const float4 a0 = *reinterpret_cast<const float4 *>(Uj + kk);
        const float4 a1 = *reinterpret_cast<const float4 *>(Uj + kk + 4);
        ua[q][0] = a0.x; ua[q][1] = a0.y; ua[q][2] = a0.z; ua[q][3] = a0.w;
        ua[q][4] = a1.x; ua[q][5] = a1.y; ua[q][6] = a1.z; ua[q][7] = a1.w;
      } else if (full) {
#pragma unroll
        for (int e = 0; e < 8; ++e) ua[q][e] = Uj[kk + e];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ua[q][e] = kk + e < k_end ? Uj[kk + e] : 0.f;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) ua[q][e] = jv ? ua[q][e] : 0.f;
    }
    f32x16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[nb][v] = 0.f;
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      if constexpr (MODE == kModeF32) {
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ua[q][e], xb[q][nb][e], acc[nb], 0, 0, 0);
      } else {
        bf16x8 ahi, alo;
        split_bf16(ua[q], ahi, alo);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, xh[q][nb], acc[nb], 0, 0, 0);
          if constexpr (MODE == kModeBF16x3) {
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, xl[q][nb], acc[nb], 0, 0, 0);
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, xh[q][nb], acc[nb], 0, 0, 0);
          }
        }
      }
    }
    if (bz > 0) __syncthreads();  // wavefront 0 has read the previous tile's sums
    if (wave > 0) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 16; ++v) red[wave - 1][nb][v][lane] = acc[nb][v];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int s = s_base + nb * 32 + i;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const float t = (acc[nb][v] + red[0][nb][v][lane]) + (red[1][nb][v][lane] + red[2][nb][v][lane]);
          const int jj = bz * 32 + 8 * (v >> 2) + 4 * kb + (v & 3);
          if (jj < r && s < b) part[((int64_t)bx * rpad + jj) * b + s] = t;
        }
      }
    }
  }
}

constexpr int kReduceThreads = 512;
__device__ __forceinline__ void corr_reduce_body(const float *__restrict__ part, int chunks, int rpad, int b, int r,
                                                 const float *__restrict__ d, float *__restrict__ out, int64_t ldo_j,
                                                 int64_t ldo_s, int bx) {
  __shared__ float red[16][kReduceOuts + 1];
  corr_reduce_block<kReduceThreads>(part, chunks, rpad, b, r, d, out, ldo_j, ldo_s, bx, red);
}

__global__ __launch_bounds__(kReduceThreads) void k_corr_reduce2(const float *__restrict__ part, int chunks, int rpad, int b,
                                                      int r, const float *__restrict__ d, float *__restrict__ out,
                                                      int64_t ldo_j, int64_t ldo_s) {
  corr_reduce_body(part, chunks, rpad, b, r, d, out, ldo_j, ldo_s, blockIdx.x);
}

// Y tile (32 samples x 32*NB signals) += U tile (32 x r) dC (r x 32*NB), with
// dC stored [j][s].  All operand loads are issued before the first matrix
// instruction (JP pairs of j at a time).  With VEC, tiles wholly inside N use
// branch-free float4 accesses of Y (clamped addresses, selects for lanes past
// the last signal); the tile crossing N takes the checked path.
template <int NB, int JP, bool VEC>
__device__ __forceinline__ void corr_apply_body(float *__restrict__ Y, int64_t ldy, int N, int b,
                                                const float *__restrict__ U, int64_t ldu, int r,
                                                const float *__restrict__ dC, int bx, int by) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, kb = lane >> 5;
  const int n0 = (bx * 4 + (threadIdx.x >> 6)) * 32;
  if (n0 >= N) return;  // whole wavefront
  const int s_base = by * 32 * NB;
  const bool full = VEC && n0 + 32 <= N;
  const bool whole = n0 + 32 <= N;  // tile inside N: no per-element guards
  f32x16 acc[NB];
  float *Ys[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int s = s_base + nb * 32 + i;
    Ys[nb] = Y + (int64_t)(s < b ? s : b - 1) * ldy;
  }
  if (full) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 t = *reinterpret_cast<const float4 *>(Ys[nb] + n0 + 8 * q + 4 * kb);
        acc[nb][4 * q + 0] = t.x;
        acc[nb][4 * q + 1] = t.y;
        acc[nb][4 * q + 2] = t.z;
        acc[nb][4 * q + 3] = t.w;
      }
  } else if (whole) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[nb][4 * q + e] = Ys[nb][n0 + 8 * q + 4 * kb + e];
  } else {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int n = n0 + 8 * q + 4 * kb + e;
          acc[nb][4 * q + e] = n < N ? Ys[nb][n] : 0.f;
        }
  }
  const int ni = n0 + i < N ? n0 + i : N - 1;
  const bool nv = n0 + i < N;
  for (int jb = 0; jb < r; jb += 2 * JP) {
    float a[JP], bv[NB][JP];
#pragma unroll
    for (int q = 0; q < JP; ++q) {
      const int j = jb + 2 * q + kb;
      const int jc = j < r ? j : r - 1;
      a[q] = U[(int64_t)jc * ldu + ni];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int s = s_base + nb * 32 + i;
        bv[nb][q] = dC[(int64_t)jc * b + (s < b ? s : b - 1)];
      }
    }
#pragma unroll
    for (int q = 0; q < JP; ++q) {
      const bool jv = jb + 2 * q + kb < r;
      a[q] = (jv && nv) ? a[q] : 0.f;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) bv[nb][q] = (jv && s_base + nb * 32 + i < b) ? bv[nb][q] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < JP; ++q) {
      if (jb + 2 * q < r) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q], bv[nb][q], acc[nb], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if (s_base + nb * 32 + i >= b) continue;
    if (full) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<float4 *>(Ys[nb] + n0 + 8 * q + 4 * kb) =
            make_float4(acc[nb][4 * q + 0], acc[nb][4 * q + 1], acc[nb][4 * q + 2], acc[nb][4 * q + 3]);
    } else if (whole) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) Ys[nb][n0 + 8 * q + 4 * kb + e] = acc[nb][4 * q + e];
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int n = n0 + 8 * q + 4 * kb + e;
          if (n < N) Ys[nb][n] = acc[nb][4 * q + e];
        }
    }
  }
}

template <int NB, int JP, bool VEC>
__global__ __launch_bounds__(256) void k_corr_apply_mfma(float *__restrict__ Y, int64_t ldy, int N, int b,
                                                         const float *__restrict__ U, int64_t ldu, int r,
                                                         const float *__restrict__ dC) {
  corr_apply_body<NB, JP, VEC>(Y, ldy, N, b, U, ldu, r, dC, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------

constexpr int kPartNB = 2;
constexpr int kPartKS = 4;      // 16-sample steps per wavefront (64 samples)
constexpr int kApplyNB = 2;
constexpr int kApplyJP = 16;

// Workgroup-level chunks of 4 * kPartKS * 16 samples.
int corr_nchunks(int64_t N, int64_t b, int r) {
  (void)b;
  (void)r;
  const int64_t kcw = 4 * kPartKS * 16;
  return (int)((N + kcw - 1) / kcw);
}

static bool aligned16(const void *p, int64_t ld) {
  return ((reinterpret_cast<uintptr_t>(p) & 15) == 0) && (ld % 4 == 0);
}

template <int MODE, bool VEC>
static void launch_partial(const char *name, dim3 grid, hipStream_t st, const float *x, int64_t ldx, int64_t N,
                           int64_t b, const float *U, int64_t ldu, int r, float *part, int rpad) {
  if (grid.z > 1) {
    const int nz = (int)grid.z;
    SLP_LAUNCH(name, (k_corr_partial_tiles<MODE, kPartNB, kPartKS, VEC>), dim3(grid.x, grid.y, 1), dim3(256), 0, st,
               x, ldx, (int)N, (int)b, U, ldu, r, part, rpad, nz);
    return;
  }
  SLP_LAUNCH(name, (k_corr_partial_mfma<MODE, kPartNB, kPartKS, VEC>), grid, dim3(256), 0, st, x, ldx, (int)N,
             (int)b, U, ldu, r, part, rpad);
}

hipError_t corr_partial_mfma(int mode, const float *x, int64_t ldx, int64_t N, int64_t b, const float *U,
                             int64_t ldu, int r, float *part, hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  const int chunks = corr_nchunks(N, b, r);
  const dim3 grid(chunks, (unsigned)((b + 32 * kPartNB - 1) / (32 * kPartNB)), (unsigned)((r + 31) / 32));
  const int rpad = corr_rpad(r);
  const bool vec = aligned16(x, ldx) && aligned16(U, ldu);
  switch (mode) {
    case kModeF32:
      if (vec) launch_partial<kModeF32, true>("corr_partial", grid, st, x, ldx, N, b, U, ldu, r, part, rpad);
      else launch_partial<kModeF32, false>("corr_partial", grid, st, x, ldx, N, b, U, ldu, r, part, rpad);
      break;
    case kModeBF16x3:
      if (vec) launch_partial<kModeBF16x3, true>("corr_partial_bf16x3", grid, st, x, ldx, N, b, U, ldu, r, part, rpad);
      else launch_partial<kModeBF16x3, false>("corr_partial_bf16x3", grid, st, x, ldx, N, b, U, ldu, r, part, rpad);
      break;
    default:
      if (vec) launch_partial<kModeBF16, true>("corr_partial_bf16", grid, st, x, ldx, N, b, U, ldu, r, part, rpad);
      else launch_partial<kModeBF16, false>("corr_partial_bf16", grid, st, x, ldx, N, b, U, ldu, r, part, rpad);
      break;
  }
  return hipGetLastError();
}

// dC stored [j][s] (leading dimension b)
hipError_t corr_reduce_mfma(const float *part, int64_t N, int64_t b, int r, const float *d, float *dC,
                            hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  const int64_t outs = (int64_t)r * b;
  SLP_LAUNCH("corr_reduce", k_corr_reduce2, dim3((unsigned)((outs + kReduceOuts - 1) / kReduceOuts)),
             dim3(kReduceThreads), 0,
             st, part,
             corr_nchunks(N, b, r), corr_rpad(r), (int)b, r, d, dC, (int64_t)b, (int64_t)1);
  return hipGetLastError();
}

hipError_t corr_sum_mfma(const float *part, int64_t N, int64_t b, int r, float *c, int64_t ldc, hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  const int64_t outs = (int64_t)r * b;
  SLP_LAUNCH("coeffs_sum", k_corr_reduce2, dim3((unsigned)((outs + kReduceOuts - 1) / kReduceOuts)),
             dim3(kReduceThreads), 0,
             st, part,
             corr_nchunks(N, b, r), corr_rpad(r), (int)b, r, nullptr, c, (int64_t)1, ldc);
  return hipGetLastError();
}

// ---- grouped launches ----

__device__ __forceinline__ int group_slot_c(const int *__restrict__ start, int m, int bid) {
  int lo = 0, hi = m;  // start[lo] <= bid < start[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= bid) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int MODE, int NB, bool VEC>
__global__ __launch_bounds__(256) void k_corr_partial_group(const GroupPlan *__restrict__ gp,
                                                            const int *__restrict__ idx,
                                                            const int *__restrict__ start, int m) {
  const int q = group_slot_c(start, m, blockIdx.x);
  const GroupPlan &P = gp[idx[q]];
  const int w = (int)blockIdx.x - start[q];
  const int gx = P.chunks, gy = (P.b + 32 * NB - 1) / (32 * NB);
  corr_partial_body<MODE, NB, kPartKS, VEC>(P.x, P.ldx, P.N, P.b, P.corr.U, P.corr.ldu, P.corr.r, P.part, P.rpad,
                                            w % gx, (w / gx) % gy, w / (gx * gy));
}

__global__ __launch_bounds__(kReduceThreads) void k_corr_reduce_group(const GroupPlan *__restrict__ gp,
                                                           const int *__restrict__ idx,
                                                           const int *__restrict__ start, int m) {
  const int q = group_slot_c(start, m, blockIdx.x);
  const GroupPlan &P = gp[idx[q]];
  corr_reduce_body(P.part, P.chunks, P.rpad, P.b, P.corr.r, P.corr.d, const_cast<float *>(P.corr.dC), (int64_t)P.b,
                   (int64_t)1, (int)blockIdx.x - start[q]);
}

int64_t group_blocks_partial(const GroupPlan &P, int nb) {
  if (P.corr.r == 0 || P.b == 0) return 0;
  return (int64_t)P.chunks * ((P.b + 32 * nb - 1) / (32 * nb)) * ((P.corr.r + 31) / 32);
}

int64_t group_blocks_reduce(const GroupPlan &P) { return ((int64_t)P.corr.r * P.b + kReduceOuts - 1) / kReduceOuts; }

template <bool VEC>
__global__ __launch_bounds__(256) void k_corr_apply_group(const GroupPlan *__restrict__ gp,
                                                          const int *__restrict__ idx,
                                                          const int *__restrict__ start, int m) {
  const int q = group_slot_c(start, m, blockIdx.x);
  const GroupPlan &P = gp[idx[q]];
  const int w = (int)blockIdx.x - start[q];
  const int gx = (P.N + 127) / 128;
  corr_apply_body<kApplyNB, kApplyJP, VEC>(P.y, P.ldy, P.N, P.b, P.corr.U, P.corr.ldu, P.corr.r, P.corr.dC, w % gx,
                                           w / gx);
}

int64_t group_blocks_apply(const GroupPlan &P) {
  if (P.corr.r == 0 || P.b == 0) return 0;
  return (int64_t)((P.N + 127) / 128) * ((P.b + 32 * kApplyNB - 1) / (32 * kApplyNB));
}

hipError_t group_corr_apply(bool vec, const GroupPlan *gp, const GroupSpan &sp, hipStream_t st) {
  if (sp.m == 0 || sp.blocks == 0) return hipSuccess;
  const dim3 grid((unsigned)sp.blocks);
  if (vec) SLP_LAUNCH("corr_apply_group", k_corr_apply_group<true>, grid, dim3(256), 0, st, gp, sp.idx, sp.start, sp.m);
  else SLP_LAUNCH("corr_apply_group", k_corr_apply_group<false>, grid, dim3(256), 0, st, gp, sp.idx, sp.start, sp.m);
  return hipGetLastError();
}

template <int MODE, int NB>
static void launch_partial_group(const char *name, bool vec, const GroupPlan *gp, const GroupSpan &sp,
                                 hipStream_t st) {
  const dim3 grid((unsigned)sp.blocks);
  if (vec) SLP_LAUNCH(name, (k_corr_partial_group<MODE, NB, true>), grid, dim3(256), 0, st, gp, sp.idx, sp.start, sp.m);
  else SLP_LAUNCH(name, (k_corr_partial_group<MODE, NB, false>), grid, dim3(256), 0, st, gp, sp.idx, sp.start, sp.m);
}

hipError_t group_corr_partial(int mode, int nb, bool vec, const GroupPlan *gp, const GroupSpan &sp,
                              hipStream_t st) {
  if (sp.m == 0 || sp.blocks == 0) return hipSuccess;
  if (nb != 1 && nb != 2) return hipErrorInvalidValue;
  if (mode == kModeF32) {
    if (nb == 2) launch_partial_group<kModeF32, 2>("corr_partial_group", vec, gp, sp, st);
    else launch_partial_group<kModeF32, 1>("corr_partial_group", vec, gp, sp, st);
  } else if (mode == kModeBF16x3) {
    if (nb == 2) launch_partial_group<kModeBF16x3, 2>("corr_partial_bf16x3_group", vec, gp, sp, st);
    else launch_partial_group<kModeBF16x3, 1>("corr_partial_bf16x3_group", vec, gp, sp, st);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t group_corr_reduce(const GroupPlan *gp, const GroupSpan &sp, hipStream_t st) {
  if (sp.m == 0 || sp.blocks == 0) return hipSuccess;
  SLP_LAUNCH("corr_reduce_group", k_corr_reduce_group, dim3((unsigned)sp.blocks), dim3(kReduceThreads), 0, st, gp,
             sp.idx,
             sp.start, sp.m);
  return hipGetLastError();
}

template <int NB>
static void launch_apply(float *y, int64_t ldy, int64_t N, int64_t b, const float *U, int64_t ldu, int r,
                         const float *dC, hipStream_t st) {
  const dim3 grid((unsigned)((N + 127) / 128), (unsigned)((b + 32 * NB - 1) / (32 * NB)));
  if (aligned16(y, ldy)) {
    SLP_LAUNCH("corr_apply", (k_corr_apply_mfma<NB, kApplyJP, true>), grid, dim3(256), 0, st, y, ldy, (int)N, (int)b,
               U, ldu, r, dC);
  } else {
    SLP_LAUNCH("corr_apply", (k_corr_apply_mfma<NB, kApplyJP, false>), grid, dim3(256), 0, st, y, ldy, (int)N, (int)b,
               U, ldu, r, dC);
  }
}

// Batches of 128 signals or more take 128 signals per wavefront (U's loads
// shared by twice the signals; 537 -> 522 us at N = 2^18, 1024 signals).
// A signal's sums do not depend on the block width, so every width (and the
// grouped launches, which keep 64) gives the same bits.
hipError_t corr_apply_mfma(float *y, int64_t ldy, int64_t N, int64_t b, const float *U, int64_t ldu, int r,
                           const float *dC, hipStream_t st) {
  if (r == 0 || b == 0) return hipSuccess;
  if (b >= 128) launch_apply<4>(y, ldy, N, b, U, ldu, r, dC, st);
  else launch_apply<kApplyNB>(y, ldy, N, b, U, ldu, r, dC, st);
  return hipGetLastError();
}

}  // namespace slp

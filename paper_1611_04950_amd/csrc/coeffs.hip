// Slepian coefficients c = S_K^T x (the compression S_K^* x of Section 1.3,
// the exact counterpart of the fast factorization) as a hand-written matrix-
// core GEMM.  S_K is N x K (every Slepian vector a column) and x is N x b;
// both run along the reduction index n, so C (K x b) = sum_n S[n][k] x[n][s].
//
// Operand images.  Each column (a Slepian vector or a signal) is cut into
// steps of 32 samples, and each step into one 128-byte line of eight 16-byte
// pieces, zero past N:
//   mode 0 (FP32):  piece p = 4 sub + 2 kb + h holds samples
//                   32 t + 16 sub + 8 kb + 4 h + (0..3), i.e. the column
//                   itself with a leading dimension rounded up to 32;
//   mode 1 (BF16 hi/lo):  piece p = 4 sub + 2 plane + kb holds the eight
//                   samples 32 t + 16 sub + 8 kb + e (e < 8) as BF16, plane 0
//                   hi = bf16(v), plane 1 lo = bf16(v - hi).
// The plan keeps S_K's image; the call stages x's.
//
// Kernel.  A workgroup (4 wavefronts) owns a 128 x 256 tile of C (Slepian
// index k x signal s) and a range of steps (split over the reduction when the
// tiles alone would not fill the chip).  Per step it moves 128 + 256 lines
// from memory into LDS (one 16-byte piece per lane, eight lanes per line:
// whole-line reads), double-buffered, with the next step's loads in flight
// in registers while a step's matrix work runs.  Wavefront w computes the
// 64 x 128 sub-tile (w % 2, w / 2) with eight 32 x 32 FP32 accumulators:
// per 16-sample substep lane (i, kb) = (lane % 32, lane / 32) reads the eight
// samples 16 sub + 8 kb + e of row i of each 32-row block, and
//   mode 0: eight v_mfma_f32_32x32x2_f32 per block pair (sample e),
//   mode 1: three v_mfma_f32_32x32x16_bf16 (hi hi, hi lo, lo hi), FP32
//           accumulation.
// In LDS piece p of row c sits at slab p, row c ^ p: the eight lanes that
// store one line hit eight different 16-byte slots, and the reads of 32
// consecutive rows stay contiguous.  Partial tiles go to a workspace, one
// per reduction split, and a fixed-order sum writes c (deterministic).
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kBM = 128;      // Slepian indices per workgroup
constexpr int kBN = 256;      // signals per workgroup
constexpr int kCfThreads = 256;
static_assert(kBM * 8 / kCfThreads == 4 && kBN * 8 / kCfThreads == 8, "pieces per lane (Stage)");
constexpr int kLine = 128;                    // bytes per column and step
constexpr int kStageA = kBM * kLine;          // the S lines of a step (16 KB)
constexpr int kStage = (kBM + kBN) * kLine;   // one step's lines (48 KB)

struct Img {
  const char *p;     // base of column 0
  int64_t stride;    // bytes between columns (Tn * 128)
  int64_t ncols;     // valid columns (loads beyond are clamped)
};

// One step's pieces in registers: four of S's lines' pieces and eight of
// x's per lane (named members, so they stay in registers).
struct Stage {
  float4 a0, a1, a2, a3, b0, b1, b2, b3, b4, b5, b6, b7;
};

// Piece p of step t of local column c of a tile whose first column starts at
// `base` (uniform): a 32-bit per-lane offset from a uniform base, so that an
// address costs one register.  Columns past the last valid one (cmax) reload
// it; those results are never stored.
__device__ __forceinline__ float4 ld_piece(const char *base, uint32_t stride, int c, int cmax, int t, int p) {
  const uint32_t cc = (uint32_t)(c < cmax ? c : cmax);
  return *reinterpret_cast<const float4 *>(base + (cc * stride + (uint32_t)t * 128u + (uint32_t)p * 16u));
}

// lane tid loads piece p = tid % 8 of lines tid / 8 + 32 j: eight lanes per
// 128-byte line
__device__ __forceinline__ void issue(const Img &A, const Img &B, int64_t k0, int64_t s0, int t, Stage &g) {
  const int tid = threadIdx.x;
  const int p = tid & 7, r = tid >> 3;
  const char *ba = A.p + k0 * A.stride, *bb = B.p + s0 * B.stride;
  const uint32_t sa = (uint32_t)A.stride, sb = (uint32_t)B.stride;
  const int ca = (int)(A.ncols - 1 - k0), cb = (int)(B.ncols - 1 - s0);
  g.a0 = ld_piece(ba, sa, r, ca, t, p);
  g.a1 = ld_piece(ba, sa, 32 + r, ca, t, p);
  g.a2 = ld_piece(ba, sa, 64 + r, ca, t, p);
  g.a3 = ld_piece(ba, sa, 96 + r, ca, t, p);
  g.b0 = ld_piece(bb, sb, r, cb, t, p);
  g.b1 = ld_piece(bb, sb, 32 + r, cb, t, p);
  g.b2 = ld_piece(bb, sb, 64 + r, cb, t, p);
  g.b3 = ld_piece(bb, sb, 96 + r, cb, t, p);
  g.b4 = ld_piece(bb, sb, 128 + r, cb, t, p);
  g.b5 = ld_piece(bb, sb, 160 + r, cb, t, p);
  g.b6 = ld_piece(bb, sb, 192 + r, cb, t, p);
  g.b7 = ld_piece(bb, sb, 224 + r, cb, t, p);
}

// Piece p of line `row` of a stage region sits at slot p ^ ((row / 2) % 8):
// the 16 rows one read of 16 lanes touches cover all 16 bank groups of two
// 128-byte rows, and the eight pieces of one line still fill the line.
__device__ __forceinline__ int slot_of(int row, int p) { return p ^ ((row >> 1) & 7); }

__device__ __forceinline__ const char *piece_at(const char *region, int row, int p) {
  return region + row * kLine + (slot_of(row, p) << 4);
}

__device__ __forceinline__ void put(char *region, int row, int p, float4 v) {
  *reinterpret_cast<float4 *>(region + row * kLine + (slot_of(row, p) << 4)) = v;
}

__device__ __forceinline__ void commit(const Stage &g, char *buf) {
  const int tid = threadIdx.x;
  const int p = tid & 7, r = tid >> 3;
  char *sa = buf;
  char *sb = buf + kStageA;
  put(sa, r, p, g.a0);
  put(sa, 32 + r, p, g.a1);
  put(sa, 64 + r, p, g.a2);
  put(sa, 96 + r, p, g.a3);
  put(sb, r, p, g.b0);
  put(sb, 32 + r, p, g.b1);
  put(sb, 64 + r, p, g.b2);
  put(sb, 96 + r, p, g.b3);
  put(sb, 128 + r, p, g.b4);
  put(sb, 160 + r, p, g.b5);
  put(sb, 192 + r, p, g.b6);
  put(sb, 224 + r, p, g.b7);
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Direct-to-LDS loads of one step: each instruction moves 8 whole lines (1 KB;
// lane L writes line c0 + L / 8, slot L % 8, so it fetches the piece that
// slot holds).  Wavefront w issues line groups w, w + 4, ... of S's 16 and
// x's 32.
__device__ __forceinline__ void dma_step(const Img &A, const Img &B, int64_t k0, int64_t s0, int t, char *stage) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int rl = lane >> 3;
  const char *ba = A.p + k0 * A.stride, *bb = B.p + s0 * B.stride;
  const uint32_t sa = (uint32_t)A.stride, sb = (uint32_t)B.stride;
  const int ca = (int)(A.ncols - 1 - k0), cb = (int)(B.ncols - 1 - s0);
  const uint32_t t128 = (uint32_t)t * 128u;
#pragma unroll
  for (int j = 0; j < kBM / 32; ++j) {
    const int grp = wave + 4 * j;
    const int c = 8 * grp + rl;
    const int p = slot_of(c, lane & 7);  // the slot map is its own inverse
    const uint32_t cc = (uint32_t)(c < ca ? c : ca);
    __builtin_amdgcn_global_load_lds(ba + (cc * sa + t128 + (uint32_t)p * 16u), (lds_void_t *)(stage + grp * 1024), 16,
                                     0, 0);
  }
#pragma unroll
  for (int j = 0; j < kBN / 32; ++j) {
    const int grp = wave + 4 * j;
    const int c = 8 * grp + rl;
    const int p = slot_of(c, lane & 7);
    const uint32_t cc = (uint32_t)(c < cb ? c : cb);
    __builtin_amdgcn_global_load_lds(bb + (cc * sb + t128 + (uint32_t)p * 16u),
                                     (lds_void_t *)(stage + kStageA + grp * 1024), 16, 0, 0);
  }
}

template <int MODE>
__device__ __forceinline__ void compute(const char *buf, f32x16 (&acc)[2][4], int wk, int ws) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, kb = lane >> 5;
  const char *sa = buf;
  const char *sb = buf + kStageA;
#pragma unroll
  for (int sub = 0; sub < 2; ++sub) {
    if constexpr (MODE == 1) {
      bf16x8 ah[2], al[2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const int row = 64 * wk + 32 * mb + i;
        const int ph = 4 * sub + kb, pl = 4 * sub + 2 + kb;
        ah[mb] = *reinterpret_cast<const bf16x8 *>(piece_at(sa, row, ph));
        al[mb] = *reinterpret_cast<const bf16x8 *>(piece_at(sa, row, pl));
      }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int row = 128 * ws + 32 * nb + i;
        const int ph = 4 * sub + kb, pl = 4 * sub + 2 + kb;
        const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(piece_at(sb, row, ph));
        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(piece_at(sb, row, pl));
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mb], bh, acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[mb], bl, acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[mb], bh, acc[mb][nb], 0, 0, 0);
        }
      }
    } else {
      float a[2][8];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const int row = 64 * wk + 32 * mb + i;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int p = 4 * sub + 2 * kb + h;
          const float4 v = *reinterpret_cast<const float4 *>(piece_at(sa, row, p));
          a[mb][4 * h + 0] = v.x;
          a[mb][4 * h + 1] = v.y;
          a[mb][4 * h + 2] = v.z;
          a[mb][4 * h + 3] = v.w;
        }
      }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int row = 128 * ws + 32 * nb + i;
        float bv[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int p = 4 * sub + 2 * kb + h;
          const float4 v = *reinterpret_cast<const float4 *>(piece_at(sb, row, p));
          bv[4 * h + 0] = v.x;
          bv[4 * h + 1] = v.y;
          bv[4 * h + 2] = v.z;
          bv[4 * h + 3] = v.w;
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int e = 0; e < 8; ++e)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mb][e], bv[e], acc[mb][nb], 0, 0, 0);
      }
    }
  }
}

// Grid: one workgroup per (tile of 128 k, tile of 256 s, reduction split),
// tiles ordered with k fastest and dealt to the eight XCDs in contiguous
// runs, so that the workgroups sharing x's lines share an L2.
template <int MODE, bool DMA>
__global__ __launch_bounds__(kCfThreads, 1) void k_coeffs(Img A, Img B, int tiles_k, int tiles_s, int splits,
                                                         int steps, int steps_per_split, float *__restrict__ out,
                                                         int64_t ldo, int64_t split_stride, int64_t K, int64_t b) {
  __shared__ __align__(16) char lds[(DMA ? 3 : 2) * kStage];
  const int G = tiles_k * tiles_s * splits;
  const int L = blockIdx.x;
  const int tile = (G & 7) ? L : (L & 7) * (G >> 3) + (L >> 3);
  const int tk = tile % tiles_k;
  const int ts = (tile / tiles_k) % tiles_s;
  const int z = tile / (tiles_k * tiles_s);
  const int64_t k0 = (int64_t)tk * kBM, s0 = (int64_t)ts * kBN;
  const int t0 = z * steps_per_split;
  const int t1 = steps < t0 + steps_per_split ? steps : t0 + steps_per_split;
  const int nt = t1 > t0 ? t1 - t0 : 0;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int wk = wave & 1, ws = wave >> 1;
  f32x16 acc[2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.f;
  if constexpr (DMA) {
    // Three LDS stages, two steps' direct-to-LDS loads in flight: step i + 2
    // is issued into the stage step i - 1 used, right after the barrier that
    // ends step i - 1's matrix work, and this wavefront's share is waited
    // for two steps later; the barrier then makes every share visible.  Past
    // the range the loads repeat the last step (unused), so every step issues
    // the same number of loads and the wait count stays fixed.  The barrier
    // is the bare instruction (a full __syncthreads would also wait for the
    // loads still in flight).
    const int tl = t0 + nt - 1;  // last step of the range (no loads when it is empty)
    static_assert((kBM + kBN) / 32 == 12, "loads per wavefront and step (the wait count)");
    if (nt > 0) {
      dma_step(A, B, k0, s0, t0, lds);
      dma_step(A, B, k0, s0, t0 + 1 <= tl ? t0 + 1 : tl, lds + kStage);
    }
    for (int i = 0; i < nt; ++i) {
      __builtin_amdgcn_s_waitcnt(12 | (7 << 4) | (15 << 8));  // vmcnt(12): step i's share has landed
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      dma_step(A, B, k0, s0, t0 + i + 2 <= tl ? t0 + i + 2 : tl, lds + ((i + 2) % 3) * kStage);
      __builtin_amdgcn_sched_barrier(0);
      compute<MODE>(lds + (i % 3) * kStage, acc, wk, ws);
    }
    // no load may still be writing LDS when the workgroup ends
    __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));
  } else {
    // Step i computes from LDS buffer i % 2 while the loads of step i + 1 are
    // in flight into registers; they are stored into the other buffer after
    // the step's matrix work, and one barrier per step orders the two.  Loads
    // are issued unconditionally (the last step reloads itself, unused): loads
    // under a branch would be waited for at the branch's end.
    Stage g;
    if (nt > 0) {
      issue(A, B, k0, s0, t0, g);
      commit(g, lds);
    }
    __syncthreads();
    for (int i = 0; i < nt; ++i) {
      char *cur = lds + (i & 1) * kStage;
      char *nxt = lds + ((i + 1) & 1) * kStage;
      issue(A, B, k0, s0, i + 1 < nt ? t0 + i + 1 : t0 + i, g);
      // keep the loads ahead of the matrix work (the scheduler would otherwise
      // sink them below it to share registers, exposing their latency)
      __builtin_amdgcn_sched_barrier(0);
      compute<MODE>(cur, acc, wk, ws);
      if (i + 1 < nt) commit(g, nxt);
      __syncthreads();
    }
  }
  // D[8 (v / 4) + 4 kb + v % 4][i] of block (mb, nb): k = k0 + 64 wk + 32 mb
  // + 8 (v / 4) + 4 kb + v % 4, s = s0 + 128 ws + 32 nb + i
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, kb = lane >> 5;
  float *o = out + (int64_t)z * split_stride;
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int64_t s = s0 + 128 * ws + 32 * nb + i;
    if (s >= b) continue;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int vg = 0; vg < 4; ++vg) {
        const int64_t k = k0 + 64 * wk + 32 * mb + 8 * vg + 4 * kb;
        if (k < K)
          *reinterpret_cast<float4 *>(o + s * ldo + k) =
              float4{acc[mb][nb][4 * vg], acc[mb][nb][4 * vg + 1], acc[mb][nb][4 * vg + 2], acc[mb][nb][4 * vg + 3]};
      }
  }
}

// c[s ldc + k] = sum over splits z (in order) of part[z][s ldp + k]
__global__ __launch_bounds__(256) void k_coeffs_sum(const float *__restrict__ part, int64_t ldp, int64_t zstride,
                                                     int splits, float *__restrict__ c, int64_t ldc, int64_t K) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t s = blockIdx.y;
  if (k >= K) return;
  float t = part[s * ldp + k];
  for (int z = 1; z < splits; ++z) t += part[(int64_t)z * zstride + s * ldp + k];
  c[s * ldc + k] = t;
}

// The BF16 hi/lo image of FP32 columns (mode 1): one 16-byte piece per thread.
__global__ __launch_bounds__(256) void k_coeffs_image_bf16(const float *__restrict__ src, int64_t lds, int64_t N,
                                                            int64_t ncols, int64_t Tn, uint4 *__restrict__ dst) {
  const int64_t total = ncols * Tn * 8;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
    const int64_t col = q / (Tn * 8);
    const int64_t t = (q >> 3) % Tn;
    const int p = (int)(q & 7);
    const int sub = p >> 2, plane = (p >> 1) & 1, kb = p & 1;
    const int64_t n0 = 32 * t + 16 * sub + 8 * kb;
    const float *col_src = src + col * lds;
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float f = n0 + e < N ? col_src[n0 + e] : 0.f;
      const __bf16 h = (__bf16)f;
      v[e] = plane ? (__bf16)(f - (float)h) : h;
    }
    dst[q] = __builtin_bit_cast(uint4, v);
  }
}

// The FP32 image (mode 0): columns copied with the leading dimension Tn * 32,
// zero past N.
__global__ __launch_bounds__(256) void k_coeffs_image_f32(const float *__restrict__ src, int64_t lds, int64_t N,
                                                           int64_t ncols, int64_t ld, float *__restrict__ dst) {
  const int64_t total = ncols * ld;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
    const int64_t col = q / ld, n = q % ld;
    dst[q] = n < N ? src[col * lds + n] : 0.f;
  }
}

unsigned grid_for(int64_t items) { return (unsigned)std::min<int64_t>((items + 255) / 256, 1 << 20); }

}  // namespace

int64_t coeffs_steps(int64_t N) { return (N + 31) / 32; }

int coeffs_splits(int64_t N, int64_t K, int64_t b) {
  const int64_t tiles = ((K + kBM - 1) / kBM) * ((b + kBN - 1) / kBN);
  const int64_t steps = coeffs_steps(N);
  // fill the 256 compute units, each split keeping at least 32 steps
  int64_t sp = std::max<int64_t>(1, (256 + tiles - 1) / tiles);
  sp = std::min<int64_t>(sp, std::max<int64_t>(1, steps / 32));
  return (int)std::min<int64_t>(sp, 64);
}

size_t coeffs_image_bytes(int64_t N, int64_t ncols) { return (size_t)ncols * (size_t)coeffs_steps(N) * 128; }

hipError_t coeffs_image(int mode, const float *src, int64_t lds, int64_t N, int64_t ncols, void *dst,
                        hipStream_t st) {
  if (ncols == 0 || N == 0) return hipSuccess;
  const int64_t Tn = coeffs_steps(N);
  if (mode == 1) {
    SLP_LAUNCH("coeffs_image_bf16x2", k_coeffs_image_bf16, dim3(grid_for(ncols * Tn * 8)), dim3(256), 0, st, src, lds,
               N, ncols, Tn, static_cast<uint4 *>(dst));
  } else {
    SLP_LAUNCH("coeffs_image_f32", k_coeffs_image_f32, dim3(grid_for(ncols * Tn * 32)), dim3(256), 0, st, src, lds,
               N, ncols, Tn * 32, static_cast<float *>(dst));
  }
  return hipGetLastError();
}

size_t coeffs_part_floats(int64_t N, int64_t K, int64_t b) {
  const int64_t ldp = (K + 3) / 4 * 4;
  return (size_t)coeffs_splits(N, K, b) * (size_t)b * (size_t)ldp;
}

hipError_t coeffs_gemm(int mode, const void *Simg, const void *Ximg, int64_t N, int64_t K, int64_t b, float *part,
                       float *c, int64_t ldc, hipStream_t st) {
  if (K == 0 || b == 0) return hipSuccess;
  if (mode != 0 && mode != 1) return hipErrorInvalidValue;
  const int64_t steps = coeffs_steps(N);
  const int tiles_k = (int)((K + kBM - 1) / kBM), tiles_s = (int)((b + kBN - 1) / kBN);
  const int splits = coeffs_splits(N, K, b);
  const int per = (int)((steps + splits - 1) / splits);
  const int64_t G = (int64_t)tiles_k * tiles_s * splits;
  if (G > 0x7fffffff || b > 65535 || steps > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t ldp = (K + 3) / 4 * 4;
  const int64_t zstride = ldp * b;
  Img A{static_cast<const char *>(Simg), steps * 128, K};
  Img B{static_cast<const char *>(Ximg), steps * 128, b};
  if (mode == 1)
    SLP_LAUNCH("coeffs_gemm_bf16x3", (k_coeffs<1, true>), dim3((unsigned)G), dim3(kCfThreads), 0, st, A, B, tiles_k, tiles_s,
               splits, (int)steps, per, part, ldp, zstride, K, b);
  else
    SLP_LAUNCH("coeffs_gemm", (k_coeffs<0, false>), dim3((unsigned)G), dim3(kCfThreads), 0, st, A, B, tiles_k, tiles_s, splits,
               (int)steps, per, part, ldp, zstride, K, b);
  SLP_LAUNCH("coeffs_sum", k_coeffs_sum, dim3((unsigned)((K + 255) / 256), (unsigned)b), dim3(256), 0, st, part, ldp,
             zstride, splits, c, ldc, K);
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

}  // namespace slp

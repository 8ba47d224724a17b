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
//   mode 1 (BF16 hi/lo):  in 16-sample substeps u of one 64-byte half-line
//                   per column, piece q = 2 plane + kb holds the eight
//                   samples 16 u + 8 kb + e (e < 8) as BF16, plane 0
//                   hi = bf16(v), plane 1 lo = bf16(v - hi); substep-major
//                   (half-line (u, col) at u ncols + col), so the half-lines
//                   of one substep that a workgroup reads are contiguous and
//                   the workgroups sharing a substep stream one region.
// The plan keeps S_K's image; the call stages x's.
//
// Kernels.  A workgroup (4 wavefronts) owns a tile of C (Slepian index k x
// signal s) and a range of steps (split over the reduction when the tiles
// alone would not fill the chip); partial tiles go to a workspace, one per
// reduction split, and a fixed-order sum writes c (deterministic).
//   mode 0 (FP32, k_coeffs_f32): 128 x 256 tiles.  Per step the workgroup
//           moves 128 + 256 lines from memory into LDS (one 16-byte piece
//           per lane, eight lanes per line: whole-line reads), double-
//           buffered, with the next step's loads in flight in registers while
//           a step's matrix work runs.  Wavefront w computes the 64 x 128
//           sub-tile (w % 2, w / 2), eight v_mfma_f32_32x32x2_f32 per 32 x 32
//           block pair and 8-sample piece.
//   mode 1 (BF16 hi/lo, k_coeffs_bf16): 256 x 256 tiles, twice the matrix
//           work per byte moved.  The lines go straight from memory into LDS
//           (direct-to-LDS loads, no registers), two stages.  Wavefront w
//           computes the 128 x 128 sub-tile (w % 2, w / 2) with sixteen
//           32 x 32 FP32 accumulators (the accumulation registers), three
//           v_mfma_f32_32x32x16_bf16 per block pair and substep (hi hi,
//           hi lo, lo hi).
// Per 16-sample substep lane (i, kb) = (lane % 32, lane / 32) reads the
// samples 16 sub + 8 kb + (0..7) of row i of each 32-row block.  In LDS
// piece p of a line sits at slot p ^ ((row / 2) % 8) of its row: the lanes
// that store one line hit eight different 16-byte slots, and a read of 16
// consecutive rows covers every bank group of two rows.
#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kBM = 128;      // Slepian indices per workgroup (FP32)
constexpr int kBM2 = 256;     // Slepian indices per workgroup (BF16 hi/lo)
constexpr int kBN = 256;      // signals per workgroup
constexpr int kCfThreads = 256;
static_assert(kBM * 8 / kCfThreads == 4 && kBN * 8 / kCfThreads == 8, "pieces per lane (Stage)");
constexpr int kLine = 128;                    // bytes per column and step
constexpr int kStageA = kBM * kLine;          // the S lines of a step (16 KB)
constexpr int kStage = (kBM + kBN) * kLine;   // one step's lines (48 KB)
constexpr int kHalf = 64;                     // BF16 image: bytes per column and substep
constexpr int kStageA2 = kBM2 * kHalf;        // BF16 tiles: the S half-lines of a substep (16 KB)
constexpr int kStage2 = (kBM2 + kBN) * kHalf; // BF16 tiles: one substep's half-lines (32 KB)
constexpr int kStages2 = 4;                   // BF16 tiles: LDS stages (three substeps in flight)

struct Img {
  const char *p;     // base of column 0
  int64_t stride;    // bytes between columns of one step (or substep)
  int64_t tstride;   // bytes between steps (or substeps) of one column
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

// BF16 tiles in LDS: a substep's 64-byte half-line of row r (pieces hi kb0,
// hi kb1, lo kb0, lo kb1) has piece q at slot q ^ ((r / 4) % 4), so that the
// 16 lanes of one read phase (16 consecutive rows, one piece) hit the 16
// bank groups of 256 bytes.
__device__ __forceinline__ int slot2(int row, int q) { return q ^ ((row >> 2) & 3); }

// Direct-to-LDS loads of one substep of a BF16 tile: each instruction fills
// 1 KB of LDS, lane L the 16 bytes at L * 16, i.e. row 16 g + L / 4, slot
// L % 4 of line group g, so the lane fetches the piece that slot holds.
// Wavefront w issues groups w, w + 4, ... of S's 16 and x's 16.  A lane's
// byte offsets within the tile do not depend on the substep, so they are
// formed once; a substep only moves the uniform bases.
struct DmaOffs {
  uint32_t a[kBM2 / 64], b[kBN / 64];
};

__device__ __forceinline__ void dma_offsets(const Img &A, const Img &B, int64_t k0, int64_t s0, DmaOffs &o) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int rl = lane >> 2;
  const uint32_t sa = (uint32_t)A.stride, sb = (uint32_t)B.stride;
  const int ca = (int)(A.ncols - 1 - k0), cb = (int)(B.ncols - 1 - s0);
#pragma unroll
  for (int j = 0; j < kBM2 / 64; ++j) {
    const int c = 16 * (wave + 4 * j) + rl;
    const int q = slot2(c, lane & 3);  // the slot map is its own inverse
    o.a[j] = (uint32_t)(c < ca ? c : ca) * sa + (uint32_t)q * 16u;
  }
#pragma unroll
  for (int j = 0; j < kBN / 64; ++j) {
    const int c = 16 * (wave + 4 * j) + rl;
    const int q = slot2(c, lane & 3);
    o.b[j] = (uint32_t)(c < cb ? c : cb) * sb + (uint32_t)q * 16u;
  }
}

// ba, bb: the tile's first S and x columns (uniform); u: the substep
__device__ __forceinline__ void dma_step(const Img &A, const Img &B, const char *ba, const char *bb, const DmaOffs &o,
                                         int u, char *stage) {
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const char *at = ba + (int64_t)u * A.tstride, *bt = bb + (int64_t)u * B.tstride;
#pragma unroll
  for (int j = 0; j < kBM2 / 64; ++j)
    __builtin_amdgcn_global_load_lds(at + o.a[j], (lds_void_t *)(stage + (wave + 4 * j) * 1024), 16, 0, 0);
#pragma unroll
  for (int j = 0; j < kBN / 64; ++j)
    __builtin_amdgcn_global_load_lds(bt + o.b[j], (lds_void_t *)(stage + kStageA2 + (wave + 4 * j) * 1024), 16, 0,
                                     0);
}

// The BF16 operands of one substep of a wavefront's 128 x 128 sub-tile:
// lane (i, kb) holds the hi and lo pieces kb of row i of each 32-row block
// (4 of S, 4 of x)
struct Ops {
  bf16x8 ah[4], al[4], bh[4], bl[4];
};

__device__ __forceinline__ const bf16x8 &piece2(const char *region, int row, int q) {
  return *reinterpret_cast<const bf16x8 *>(region + row * kHalf + (slot2(row, q) << 4));
}

__device__ __forceinline__ void load_ops(const char *stage, int wk, int ws, Ops &o) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, kb = lane >> 5;
  const char *sa = stage;
  const char *sb = stage + kStageA2;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int row = 128 * wk + 32 * mb + i;
    o.ah[mb] = piece2(sa, row, kb);
    o.al[mb] = piece2(sa, row, 2 + kb);
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int row = 128 * ws + 32 * nb + i;
    o.bh[nb] = piece2(sb, row, kb);
    o.bl[nb] = piece2(sb, row, 2 + kb);
  }
}

// hi hi, hi lo, lo hi per block pair
__device__ __forceinline__ void mma_ops(const Ops &o, f32x16 (&acc)[4][4]) {
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[mb], o.bh[nb], acc[mb][nb], 0, 0, 0);
      acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[mb], o.bl[nb], acc[mb][nb], 0, 0, 0);
      acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.al[mb], o.bh[nb], acc[mb][nb], 0, 0, 0);
    }
}

// The FP32 matrix work of one step of a 128 x 256 tile: wavefront (wk, ws)
// takes rows 64 wk.. of S's lines and 128 ws.. of x's, eight
// v_mfma_f32_32x32x2_f32 per block pair and 8-sample piece.
__device__ __forceinline__ void compute_f32(const char *buf, f32x16 (&acc)[2][4], int wk, int ws) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, kb = lane >> 5;
  const char *sa = buf;
  const char *sb = buf + kStageA;
#pragma unroll
  for (int sub = 0; sub < 2; ++sub) {
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

// A workgroup's tile and step range: tiles ordered with k fastest and dealt
// to the eight XCDs in contiguous runs, so that the workgroups sharing x's
// lines share an L2.
struct TileRange {
  int64_t k0, s0;
  int z, t0, nt;
};

__device__ __forceinline__ TileRange tile_range(int BM, int tiles_k, int tiles_s, int splits, int steps, int per) {
  const int G = tiles_k * tiles_s * splits;
  const int L = blockIdx.x;
  const int tile = (G & 7) ? L : (L & 7) * (G >> 3) + (L >> 3);
  const int tk = tile % tiles_k;
  const int ts = (tile / tiles_k) % tiles_s;
  TileRange r;
  r.z = tile / (tiles_k * tiles_s);
  r.k0 = (int64_t)tk * BM;
  r.s0 = (int64_t)ts * kBN;
  r.t0 = r.z * per;
  const int t1 = steps < r.t0 + per ? steps : r.t0 + per;
  r.nt = t1 > r.t0 ? t1 - r.t0 : 0;
  return r;
}

// The accumulators of a wavefront's MB x 4 blocks of 32 x 32 to split z's
// partial tile: D[8 (v / 4) + 4 kb + v % 4][i] of block (mb, nb) is
// k = k0 + rows + 32 mb + 8 (v / 4) + 4 kb + v % 4, s = s0 + cols + 32 nb + i
template <int MB>
__device__ __forceinline__ void store_tile(const f32x16 (&acc)[MB][4], float *__restrict__ o, int64_t ldo, int64_t k0,
                                           int64_t s0, int64_t K, int64_t b) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, kb = lane >> 5;
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int64_t s = s0 + 32 * nb + i;
    if (s >= b) continue;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int vg = 0; vg < 4; ++vg) {
        const int64_t k = k0 + 32 * mb + 8 * vg + 4 * kb;
        if (k < K)
          *reinterpret_cast<float4 *>(o + s * ldo + k) =
              float4{acc[mb][nb][4 * vg], acc[mb][nb][4 * vg + 1], acc[mb][nb][4 * vg + 2], acc[mb][nb][4 * vg + 3]};
      }
  }
}

// FP32 operands, 128 x 256 tiles, register-staged: step i computes from LDS
// buffer i % 2 while the loads of step i + 1 are in flight into registers;
// they are stored into the other buffer after the step's matrix work, and
// one barrier per step orders the two.  Loads are issued unconditionally (the
// last step reloads itself, unused): loads under a branch would be waited for
// at the branch's end.
__global__ __launch_bounds__(kCfThreads, 1) void k_coeffs_f32(Img A, Img B, int tiles_k, int tiles_s, int splits,
                                                             int steps, int per, float *__restrict__ out, int64_t ldo,
                                                             int64_t split_stride, int64_t K, int64_t b) {
  __shared__ __align__(16) char lds[2 * kStage];
  const TileRange tr = tile_range(kBM, tiles_k, tiles_s, splits, steps, per);
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int wk = wave & 1, ws = wave >> 1;
  f32x16 acc[2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.f;
  Stage g;
  if (tr.nt > 0) {
    issue(A, B, tr.k0, tr.s0, tr.t0, g);
    commit(g, lds);
  }
  __syncthreads();
  for (int i = 0; i < tr.nt; ++i) {
    char *cur = lds + (i & 1) * kStage;
    char *nxt = lds + ((i + 1) & 1) * kStage;
    issue(A, B, tr.k0, tr.s0, i + 1 < tr.nt ? tr.t0 + i + 1 : tr.t0 + i, g);
    // keep the loads ahead of the matrix work (the scheduler would otherwise
    // sink them below it to share registers, exposing their latency)
    __builtin_amdgcn_sched_barrier(0);
    compute_f32(cur, acc, wk, ws);
    if (i + 1 < tr.nt) commit(g, nxt);
    __syncthreads();
  }
  store_tile<2>(acc, out + (int64_t)tr.z * split_stride, ldo, tr.k0 + 64 * wk, tr.s0 + 128 * ws, K, b);
}

// BF16 hi/lo operands, 256 x 256 tiles, in substeps of 16 samples (one
// half-line per column), four LDS stages filled by direct-to-LDS loads.
// Before barrier B(u) each wavefront waits for its own loads of substep u
// (vmcnt(16): only those of u + 1 and u + 2 may still be in flight) and for
// its LDS reads of substep u - 1 (lgkmcnt(0)); after it, substep u's lines
// are visible to all and every wavefront is done reading substep u - 1's
// stage, into which substep u + 3's loads then go.  A substep's operands are
// read from LDS during the previous substep's matrix work.  Past the range
// the loads repeat the last substep (unused), so every substep issues the
// same number of loads and the wait count stays fixed.  The barrier is the
// bare instruction (a full __syncthreads would also wait for the loads in
// flight).
__global__ __launch_bounds__(kCfThreads, 1) void k_coeffs_bf16(Img A, Img B, int tiles_k, int tiles_s, int splits,
                                                              int steps, int per, float *__restrict__ out,
                                                              int64_t ldo, int64_t split_stride, int64_t K,
                                                              int64_t b) {
  __shared__ __align__(16) char lds[kStages2 * kStage2];
  const TileRange tr = tile_range(kBM2, tiles_k, tiles_s, splits, steps, per);
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int wk = wave & 1, ws = wave >> 1;
  f32x16 acc[4][4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[mb][nb][v] = 0.f;
  // the split's substeps u0 .. u0 + nu - 1 (two per 32-sample step)
  const int nu = 2 * tr.nt, u0 = 2 * tr.t0;
  const int ul = u0 + nu - 1;  // last substep of the range (no loads when it is empty)
  static_assert((kBM2 + kBN) / 16 / 4 == 8, "loads per wavefront and substep (the wait count)");
  const char *ba = A.p + tr.k0 * A.stride, *bb = B.p + tr.s0 * B.stride;
  DmaOffs dof;
  dma_offsets(A, B, tr.k0, tr.s0, dof);
  Ops o0, o1;
  if (nu > 0) {
#pragma unroll
    for (int k = 0; k < kStages2 - 1; ++k) dma_step(A, B, ba, bb, dof, u0 + k <= ul ? u0 + k : ul, lds + k * kStage2);
    __builtin_amdgcn_s_waitcnt(0 | (1 << 14) | (7 << 4) | (15 << 8));  // vmcnt(16): substep u0 has landed
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    dma_step(A, B, ba, bb, dof, u0 + 3 <= ul ? u0 + 3 : ul, lds + 3 * kStage2);
    load_ops(lds, wk, ws, o0);
  }
  // substep i's matrix work from cur, with substep i + 1's operands read
  // into nxt first; the scheduling barriers keep those reads ahead of the
  // matrix work that covers their latency
  auto substep = [&](int i, const Ops &cur, Ops &nxt) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0 | (1 << 14) | (7 << 4) | (0 << 8));  // vmcnt(16), lgkmcnt(0)
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    dma_step(A, B, ba, bb, dof, u0 + i + 4 <= ul ? u0 + i + 4 : ul, lds + (i & 3) * kStage2);
    load_ops(lds + ((i + 1) & 3) * kStage2, wk, ws, nxt);
    __builtin_amdgcn_sched_barrier(0);
    mma_ops(cur, acc);
  };
  // nu is even (two substeps per step): pairs of substeps with the operand
  // sets swapping roles, the last substep peeled
  for (int i = 0; i + 2 < nu; i += 2) {
    substep(i, o0, o1);
    substep(i + 1, o1, o0);
  }
  if (nu > 0) {
    substep(nu - 2, o0, o1);
    __builtin_amdgcn_sched_barrier(0);
    mma_ops(o1, acc);
  }
  // no load may still be writing LDS when the workgroup ends
  __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));
  store_tile<4>(acc, out + (int64_t)tr.z * split_stride, ldo, tr.k0 + 128 * wk, tr.s0 + 128 * ws, K, b);
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

// The BF16 hi/lo image of FP32 columns (mode 1), substep-major: one thread
// per (substep u, column), consecutive threads on consecutive columns, so a
// thread reads the column's 16 samples 16 u .. 16 u + 15 (64 bytes) and the
// threads' half-lines (u ncols + col) fill consecutive memory; pieces
// q = 2 plane + kb (hi kb 0, hi kb 1, lo kb 0, lo kb 1).
__global__ __launch_bounds__(256) void k_coeffs_image_bf16(const float *__restrict__ src, int64_t lds, int64_t N,
                                                            int64_t ncols, int64_t Tu, uint4 *__restrict__ dst) {
  const int64_t total = ncols * Tu;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
    const int64_t u = q / ncols, col = q % ncols;
    const int64_t n0 = 16 * u;
    const float *s = src + col * lds + n0;
    float v[16];
    if (n0 + 16 <= N && (reinterpret_cast<uintptr_t>(s) & 15) == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 f = reinterpret_cast<const float4 *>(s)[k];
        v[4 * k] = f.x;
        v[4 * k + 1] = f.y;
        v[4 * k + 2] = f.z;
        v[4 * k + 3] = f.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = n0 + e < N ? s[e] : 0.f;
    }
    bf16x8 h[2], l[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float f = v[8 * kb + e];
        const __bf16 hi = (__bf16)f;
        h[kb][e] = hi;
        l[kb][e] = (__bf16)(f - (float)hi);
      }
    uint4 *d = dst + 4 * q;
    d[0] = __builtin_bit_cast(uint4, h[0]);
    d[1] = __builtin_bit_cast(uint4, h[1]);
    d[2] = __builtin_bit_cast(uint4, l[0]);
    d[3] = __builtin_bit_cast(uint4, l[1]);
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

int coeffs_splits(int mode, int64_t N, int64_t K, int64_t b) {
  const int64_t bm = mode ? kBM2 : kBM;
  const int64_t tiles = ((K + bm - 1) / bm) * ((b + kBN - 1) / kBN);
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
    SLP_LAUNCH("coeffs_image_bf16x2", k_coeffs_image_bf16, dim3(grid_for(ncols * Tn * 2)), dim3(256), 0, st, src, lds,
               N, ncols, 2 * Tn, static_cast<uint4 *>(dst));
  } else {
    SLP_LAUNCH("coeffs_image_f32", k_coeffs_image_f32, dim3(grid_for(ncols * Tn * 32)), dim3(256), 0, st, src, lds,
               N, ncols, Tn * 32, static_cast<float *>(dst));
  }
  return hipGetLastError();
}

size_t coeffs_part_floats(int64_t N, int64_t K, int64_t b) {
  const int64_t ldp = (K + 3) / 4 * 4;
  const int sp = std::max(coeffs_splits(0, N, K, b), coeffs_splits(1, N, K, b));
  return (size_t)sp * (size_t)b * (size_t)ldp;
}

hipError_t coeffs_gemm(int mode, const void *Simg, const void *Ximg, int64_t N, int64_t K, int64_t b, float *part,
                       float *c, int64_t ldc, hipStream_t st) {
  if (K == 0 || b == 0) return hipSuccess;
  if (mode != 0 && mode != 1) return hipErrorInvalidValue;
  const int64_t steps = coeffs_steps(N);
  const int64_t bm = mode ? kBM2 : kBM;
  const int tiles_k = (int)((K + bm - 1) / bm), tiles_s = (int)((b + kBN - 1) / kBN);
  const int splits = coeffs_splits(mode, N, K, b);
  const int per = (int)((steps + splits - 1) / splits);
  const int64_t G = (int64_t)tiles_k * tiles_s * splits;
  if (G > 0x7fffffff || b > 65535 || steps > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t ldp = (K + 3) / 4 * 4;
  const int64_t zstride = ldp * b;
  // mode 0: column-major images (column stride, step stride); mode 1:
  // substep-major (column stride, substep stride)
  Img A{static_cast<const char *>(Simg), mode ? 64 : steps * 128, mode ? K * 64 : 128, K};
  Img B{static_cast<const char *>(Ximg), mode ? 64 : steps * 128, mode ? b * 64 : 128, b};
  if (mode == 1)
    SLP_LAUNCH("coeffs_gemm_bf16x3", k_coeffs_bf16, dim3((unsigned)G), dim3(kCfThreads), 0, st, A, B, tiles_k,
               tiles_s, splits, (int)steps, per, part, ldp, zstride, K, b);
  else
    SLP_LAUNCH("coeffs_gemm", k_coeffs_f32, dim3((unsigned)G), dim3(kCfThreads), 0, st, A, B, tiles_k, tiles_s,
               splits, (int)steps, per, part, ldp, zstride, K, b);
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

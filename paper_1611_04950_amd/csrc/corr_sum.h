// Fixed-order sum of the correction's chunk partials (C = U^T x summed over
// sample chunks, then dC = d (.) C; Corollary 2), shared by the standalone
// sum kernel and the row pass that carries it.
//
// A workgroup owns the 32 outputs o = 32 bx + og (o = j b + s, one whole
// 128-byte line of every chunk's partials).  Sixteen lane groups cg sum chunks
// cg, cg + 16, ... (eight loads in flight per round, added pairwise in a
// fixed order), then the sixteen group sums are added in order through LDS.
// With NT threads each thread plays 16 / (NT / 32) of the lane groups in
// turn, so the arithmetic, and the result, do not depend on NT.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace slp {

constexpr int kReduceOuts = 32;

template <int NT>
__device__ __forceinline__ void corr_reduce_block(const float *__restrict__ part, int chunks, int rpad, int b, int r,
                                                  const float *__restrict__ d, float *__restrict__ out,
                                                  int64_t ldo_j, int64_t ldo_s, int bx,
                                                  float (*__restrict__ red)[kReduceOuts + 1]) {
  static_assert(NT % 32 == 0 && 16 % (NT / 32) == 0, "lane groups");
  constexpr int GPT = 16 / (NT / 32);  // lane groups per thread
  const int og = threadIdx.x & 31, tg = threadIdx.x >> 5;
  const int64_t o = (int64_t)bx * kReduceOuts + og;  // o = j * b + s
  const bool valid = o < (int64_t)r * b;
  const int j = valid ? (int)(o / b) : 0, s = valid ? (int)(o % b) : 0;
  const int64_t stride = (int64_t)rpad * b;
  const float *pp = part + (int64_t)j * b + s;
#pragma unroll
  for (int h = 0; h < GPT; ++h) {
    const int cg = tg + (NT / 32) * h;
    float acc = 0.f;
    for (int c0 = cg; c0 < chunks; c0 += 128) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = c0 + 16 * e;
        v[e] = c < chunks ? pp[(int64_t)c * stride] : 0.f;
      }
      acc += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
    red[cg][og] = acc;
  }
  __syncthreads();
  if (tg == 0 && valid) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][og];
    out[(int64_t)j * ldo_j + (int64_t)s * ldo_s] = d ? d[j] * t : t;
  }
}

// Workgroups of the sum over r x b outputs.
inline int64_t corr_reduce_blocks(int r, int64_t b) { return ((int64_t)r * b + kReduceOuts - 1) / kReduceOuts; }

}  // namespace slp

// In-register DFTs of small power-of-two sizes with compile-time twiddles.
//
// dft<N, DIR>(a) replaces a[0..N) by its DFT (DIR = -1: exp(-2 pi i nk/N),
// +1: the unnormalised inverse).  Sizes above 8 are split Cooley-Tukey style,
// N = P * Q: length-Q DFTs over the stride-P subsequences, twiddles
// W_N^{n1 k1}, then length-P DFTs, output index k1 + Q k2.  Every index is a
// compile-time constant after unrolling, so the data stays in registers and
// multiplications by 1, -1, +-i and (1 +- i)/sqrt2 are removed at compile time.
#pragma once

#include "common.h"

namespace slp {
namespace reg {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Taylor series on |x| <= pi/4 (converged well below double rounding).
constexpr double sin_small(double x) {
  double t = x, s = x;
  for (int i = 1; i < 16; ++i) {
    t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
constexpr double cos_small(double x) {
  double t = 1.0, s = 1.0;
  for (int i = 1; i < 16; ++i) {
    t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}

// cos and sin of 2 pi e / n with the angle reduced exactly in integers:
// quadrant q and remainder rr (angle = q pi/2 + (pi/2) rr/n), and the
// complementary angle when rr/n > 1/2.
constexpr void cos_sin_2pi(int e, int n, double &c, double &s) {
  e %= n;
  if (e < 0) e += n;
  const int q = (4 * e) / n;
  const int rr = 4 * e - q * n;
  double ca = 0.0, sa = 0.0;
  if (2 * rr <= n) {
    const double a = (kPi / 2.0) * (double)rr / (double)n;
    ca = cos_small(a);
    sa = sin_small(a);
  } else {
    const double b = (kPi / 2.0) * (double)(n - rr) / (double)n;
    ca = sin_small(b);
    sa = cos_small(b);
  }
  switch (q) {
    case 0: c = ca; s = sa; break;
    case 1: c = -sa; s = ca; break;
    case 2: c = -ca; s = -sa; break;
    default: c = sa; s = -ca; break;
  }
}

template <int N>
struct TwTable {
  double c[N], s[N];
  constexpr TwTable() : c(), s() {
    for (int e = 0; e < N; ++e) cos_sin_2pi(e, N, c[e], s[e]);
  }
};
template <int N>
inline constexpr TwTable<N> kTw{};

template <int DIR, typename R>
__host__ __device__ __forceinline__ cpx<R> mul_i(cpx<R> a) {  // a * (DIR i)
  return DIR < 0 ? cpx<R>{a.y, -a.x} : cpx<R>{-a.y, a.x};
}

// v * exp(DIR 2 pi i e / N) for a compile-time e (after unrolling).
template <int N, int DIR, typename R>
__host__ __device__ __forceinline__ cpx<R> mul_tw(cpx<R> v, int e) {
  e %= N;
  if (e == 0) return v;
  if (4 * e == N) return mul_i<DIR>(v);
  if (2 * e == N) return cpx<R>{-v.x, -v.y};
  if (4 * e == 3 * N) return mul_i<-DIR>(v);
  const R c = (R)kTw<N>.c[e];
  const R s = (R)(DIR * kTw<N>.s[e]);
  return cpx<R>{v.x * c - v.y * s, v.x * s + v.y * c};
}

template <int N, int DIR, typename R>
__host__ __device__ __forceinline__ void dft(cpx<R> *a);

template <int DIR, typename R>
__host__ __device__ __forceinline__ void dft2(cpx<R> *a) {
  const cpx<R> t = a[0];
  a[0] = t + a[1];
  a[1] = t - a[1];
}

template <int DIR, typename R>
__host__ __device__ __forceinline__ void dft4(cpx<R> *a) {
  const cpx<R> t0 = a[0] + a[2], t1 = a[0] - a[2];
  const cpx<R> t2 = a[1] + a[3], t3 = mul_i<DIR>(a[1] - a[3]);
  a[0] = t0 + t2;
  a[2] = t0 - t2;
  a[1] = t1 + t3;
  a[3] = t1 - t3;
}

template <int DIR, typename R>
__host__ __device__ __forceinline__ void dft8(cpx<R> *a) {
  cpx<R> e[4] = {a[0], a[2], a[4], a[6]};
  cpx<R> o[4] = {a[1], a[3], a[5], a[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  const cpx<R> o1 = mul_tw<8, DIR>(o[1], 1);
  const cpx<R> o2 = mul_i<DIR>(o[2]);
  const cpx<R> o3 = mul_tw<8, DIR>(o[3], 3);
  a[0] = e[0] + o[0];
  a[4] = e[0] - o[0];
  a[1] = e[1] + o1;
  a[5] = e[1] - o1;
  a[2] = e[2] + o2;
  a[6] = e[2] - o2;
  a[3] = e[3] + o3;
  a[7] = e[3] - o3;
}

template <int P, int Q, int DIR, typename R>
__host__ __device__ __forceinline__ void dft_ct(cpx<R> *a) {
  constexpr int N = P * Q;
  cpx<R> A[P][Q];
#pragma unroll
  for (int n1 = 0; n1 < P; ++n1) {
    cpx<R> b[Q];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) b[n2] = a[n1 + P * n2];
    dft<Q, DIR>(b);
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) A[n1][k1] = mul_tw<N, DIR>(b[k1], n1 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < Q; ++k1) {
    cpx<R> c[P];
#pragma unroll
    for (int n1 = 0; n1 < P; ++n1) c[n1] = A[n1][k1];
    dft<P, DIR>(c);
#pragma unroll
    for (int k2 = 0; k2 < P; ++k2) a[k1 + Q * k2] = c[k2];
  }
}

template <int N, int DIR, typename R>
__host__ __device__ __forceinline__ void dft(cpx<R> *a) {
  if constexpr (N == 1) {
  } else if constexpr (N == 2) {
    dft2<DIR>(a);
  } else if constexpr (N == 4) {
    dft4<DIR>(a);
  } else if constexpr (N == 8) {
    dft8<DIR>(a);
  } else if constexpr (N == 16) {
    dft_ct<4, 4, DIR>(a);
  } else if constexpr (N == 32) {
    dft_ct<8, 4, DIR>(a);
  } else if constexpr (N == 64) {
    dft_ct<8, 8, DIR>(a);
  } else {
    static_assert(N <= 64, "in-register DFT size");
  }
}

}  // namespace reg
}  // namespace slp

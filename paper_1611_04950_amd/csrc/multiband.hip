// Multiband (modulated) Slepian dictionaries (Section 2.3): the projection of
// a real signal onto the union of the Slepian subspaces modulated to band
// centres f_i, each band [f_i - W, f_i + W], approximated by the sum of the
// per-band fast projections
//     y = sum_i w_i Re(E_{f_i} P~ E_{f_i}^* x),   E_f = diag(exp(2 pi i f n)),
// w_i = 2 for f_i > 0 (the band pair +-f_i of a real signal), 1 for f_i = 0.
// Demodulation writes the real and imaginary parts of E_{f_i}^* x_s as two
// adjacent signals, so the product's pair packing transforms them as one
// complex signal (B is real); remodulation takes the real part and sums the
// bands.  Phases are reduced in FP64 (f n mod 1) before the sine and cosine.
#include "common.h"
#include "kernels.h"
#include "trace.h"

namespace slp {

__device__ __forceinline__ void band_phase(double f, int64_t n, double &c, double &s) {
  const double t = f * (double)n;
  const double fr = t - floor(t);  // f n mod 1
  sincospi(2.0 * fr, &s, &c);
}

// z[2 (i b + s)][n] = x_s[n] cos(2 pi f_i n), z[2 (i b + s) + 1][n] = -x_s[n] sin(2 pi f_i n)
__global__ __launch_bounds__(256) void k_demod(const float *__restrict__ x, int64_t ldx, int N, int b, BandSet bs,
                                               float *__restrict__ z, int64_t ldz) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y, i = blockIdx.z;
  if (n >= N) return;
  double c, sn;
  band_phase(bs.f[i], n, c, sn);
  const double v = x[(int64_t)s * ldx + n];
  const int64_t q = 2 * ((int64_t)i * b + s);
  z[q * ldz + n] = (float)(v * c);
  z[(q + 1) * ldz + n] = (float)(-v * sn);
}

// y_s[n] = sum_i w_i (cos(2 pi f_i n) p[2 (i b + s)][n] - sin(2 pi f_i n) p[2 (i b + s) + 1][n])
__global__ __launch_bounds__(256) void k_remod(const float *__restrict__ p, int64_t ldp, int N, int b, BandSet bs,
                                               float *__restrict__ y, int64_t ldy) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (n >= N) return;
  double acc = 0.0;
  for (int i = 0; i < bs.J; ++i) {
    double c, sn;
    band_phase(bs.f[i], n, c, sn);
    const int64_t q = 2 * ((int64_t)i * b + s);
    const double w = bs.f[i] > 0.0 ? 2.0 : 1.0;
    acc += w * (c * (double)p[q * ldp + n] - sn * (double)p[(q + 1) * ldp + n]);
  }
  y[(int64_t)s * ldy + n] = (float)acc;
}

hipError_t band_demod(const float *x, int64_t ldx, int64_t N, int64_t b, const BandSet &bs, float *z, int64_t ldz,
                      hipStream_t st) {
  if (N == 0 || b == 0 || bs.J == 0) return hipSuccess;
  if (b > 65535 || bs.J > kMaxBands) return hipErrorInvalidValue;
  SLP_LAUNCH("band_demod", k_demod, dim3((unsigned)((N + 255) / 256), (unsigned)b, (unsigned)bs.J), dim3(256), 0, st,
             x, ldx, (int)N, (int)b, bs, z, ldz);
  return hipGetLastError();
}

hipError_t band_remod(const float *p, int64_t ldp, int64_t N, int64_t b, const BandSet &bs, float *y, int64_t ldy,
                      hipStream_t st) {
  if (N == 0 || b == 0) return hipSuccess;
  if (b > 65535 || bs.J > kMaxBands) return hipErrorInvalidValue;
  SLP_LAUNCH("band_remod", k_remod, dim3((unsigned)((N + 255) / 256), (unsigned)b), dim3(256), 0, st, p, ldp,
             (int)N, (int)b, bs, y, ldy);
  return hipGetLastError();
}

}  // namespace slp

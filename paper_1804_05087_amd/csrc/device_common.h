// Device helpers shared by the forward and adjoint kernels: complex
// arithmetic on HIP vector types and the batched in-LDS Stockham FFT.
#pragma once

#include <hip/hip_runtime.h>

#include "sp_internal.h"

namespace sp {

template <typename R>
struct V2;
template <>
struct V2<double> {
  using T = double2;
};
template <>
struct V2<float> {
  using T = float2;
};

__device__ inline double2 mk(double a, double b) { return make_double2(a, b); }
__device__ inline float2 mk(float a, float b) { return make_float2(a, b); }
__device__ inline double2 cadd(double2 a, double2 b) { return mk(a.x + b.x, a.y + b.y); }
__device__ inline float2 cadd(float2 a, float2 b) { return mk(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return mk(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cmul(float2 a, float2 b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cscale(double2 a, double s) { return mk(a.x * s, a.y * s); }
__device__ inline float2 cscale(float2 a, float s) { return mk(a.x * s, a.y * s); }
__device__ inline double2 conjc(double2 a) { return mk(a.x, -a.y); }
__device__ inline float2 conjc(float2 a) { return mk(a.x, -a.y); }
// s * i * a for s = +-1
__device__ inline double2 sidot(double2 a, double s) { return mk(-s * a.y, s * a.x); }
__device__ inline float2 sidot(float2 a, float s) { return mk(-s * a.y, s * a.x); }

template <typename R>
__device__ inline typename V2<R>::T to_r2(double2 a) {
  return mk((R)a.x, (R)a.y);
}

// ---------------------------------------------------------------------------
// Batched in-LDS Stockham FFT of nl lines of length P (line l at a[l*P]).
// Mixed radix 2/3/4 with the factor list of `pl`; tw[q] = exp(-2 pi i q / P).
// sign = -1: forward (unscaled), +1: inverse (unscaled). Returns the buffer
// holding the result (a or b). Must be called by the whole block.
// ---------------------------------------------------------------------------
template <typename R>
__device__ typename V2<R>::T* lds_fft(typename V2<R>::T* a, typename V2<R>::T* b, int nl,
                                      const FFTPlan1D& pl, const typename V2<R>::T* tw,
                                      R sign) {
  using C = typename V2<R>::T;
  const int P = pl.P;
  int Ns = 1;
  for (int s = 0; s < pl.nrad; ++s) {
    const int Rd = pl.rad[s];
    const int nb = P / Rd;
    const int tstride = P / (Ns * Rd);
    for (int t = threadIdx.x; t < nl * nb; t += blockDim.x) {
      const int l = t / nb;
      const int j = t - l * nb;
      const C* x = a + l * P;
      C* y = b + l * P;
      const int k = j % Ns;
      C v[4];
      for (int r = 0; r < Rd; ++r) v[r] = x[j + r * nb];
      if (Ns > 1) {
        for (int r = 1; r < Rd; ++r) {
          C w = tw[(k * r * tstride) % P];
          if (sign > 0) w = conjc(w);
          v[r] = cmul(v[r], w);
        }
      }
      C o[4];
      if (Rd == 2) {
        o[0] = cadd(v[0], v[1]);
        o[1] = csub(v[0], v[1]);
      } else if (Rd == 3) {
        const R h = (R)0.86602540378443864676;  // sqrt(3)/2
        C t1 = cadd(v[1], v[2]);
        C d = csub(v[1], v[2]);
        C m = csub(v[0], cscale(t1, (R)0.5));
        C e = sidot(cscale(d, h), sign);
        o[0] = cadd(v[0], t1);
        o[1] = cadd(m, e);
        o[2] = csub(m, e);
      } else {  // 4
        C s0 = cadd(v[0], v[2]);
        C s1 = csub(v[0], v[2]);
        C s2 = cadd(v[1], v[3]);
        C s3 = sidot(csub(v[1], v[3]), sign);
        o[0] = cadd(s0, s2);
        o[2] = csub(s0, s2);
        o[1] = cadd(s1, s3);
        o[3] = csub(s1, s3);
      }
      const int base = (j / Ns) * Ns * Rd + k;
      for (int r = 0; r < Rd; ++r) y[base + r * Ns] = o[r];
    }
    __syncthreads();
    C* tmp = a;
    a = b;
    b = tmp;
    Ns *= Rd;
  }
  return a;
}

}  // namespace sp

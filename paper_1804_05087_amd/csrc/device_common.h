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

// The workgroups of a launch are handed to the chip's 8 XCDs in turn
// (workgroup b to XCD b mod 8), and each XCD has its own L2. xcd_order maps the
// hardware workgroup index to a logical one so that every XCD receives one
// contiguous range of logical indices (a bijection on [0, nb)): workgroups
// whose data share cache lines then share an L2.
__device__ inline int xcd_order(int b, int nb) {
  constexpr int G = 8;
  const int x = b % G;
  const int q = nb / G;
  const int r = nb - q * G;
  return x * q + (x < r ? x : r) + b / G;
}

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


// Block-cooperative copy into LDS with the global loads of up to MAXE elements
// per thread issued before any LDS store (LDS pointers are generic here, so
// the compiler would otherwise keep each load/store pair in order).
// load(t) -> value, store(t, value); t = 0 .. total-1.
template <int MAXE, typename T, typename LoadF, typename StoreF>
__device__ inline void staged_copy(int total, LoadF load, StoreF store) {
  const int nt = blockDim.x;
  for (int base = 0; base < total; base += MAXE * nt) {
    T v[MAXE];
#pragma unroll
    for (int q = 0; q < MAXE; ++q) {
      const int t = base + q * nt + (int)threadIdx.x;
      if (t < total) v[q] = load(t);
    }
#pragma unroll
    for (int q = 0; q < MAXE; ++q) {
      const int t = base + q * nt + (int)threadIdx.x;
      if (t < total) store(t, v[q]);
    }
  }
}

// ---------------------------------------------------------------------------
// Compile-time-length variant: the radix sequence of P is fixed, so every
// index computation folds to constants; twiddles come from a table tw[q] =
// exp(-2 pi i q / P) (staged in LDS by the caller). Radix 2, 3, 4, 8.
// ---------------------------------------------------------------------------
template <typename C, typename R>
__device__ inline void bfly4(C* v, R sign) {
  const C s0 = cadd(v[0], v[2]);
  const C s1 = csub(v[0], v[2]);
  const C s2 = cadd(v[1], v[3]);
  const C s3 = sidot(csub(v[1], v[3]), sign);
  v[0] = cadd(s0, s2);
  v[2] = csub(s0, s2);
  v[1] = cadd(s1, s3);
  v[3] = csub(s1, s3);
}

template <typename C, typename R>
__device__ inline void bfly(C* v, int Rd, R sign) {
  if (Rd == 2) {
    const C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (Rd == 3) {
    const R h = (R)0.86602540378443864676;  // sqrt(3)/2
    const C t1 = cadd(v[1], v[2]);
    const C d = csub(v[1], v[2]);
    const C m = csub(v[0], cscale(t1, (R)0.5));
    const C e = sidot(cscale(d, h), sign);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, e);
    v[2] = csub(m, e);
  } else if (Rd == 4) {
    bfly4<C, R>(v, sign);
  } else {  // 8: decimation in frequency, then two radix-4
    const R c = (R)0.70710678118654752440;  // sqrt(1/2)
    C s[4], d[4];
    for (int k = 0; k < 4; ++k) {
      s[k] = cadd(v[k], v[k + 4]);
      d[k] = csub(v[k], v[k + 4]);
    }
    // d_k *= W8^k, W8 = exp(sign 2 pi i / 8)
    d[1] = cmul(d[1], mk(c, sign * c));
    d[2] = sidot(d[2], sign);
    d[3] = cmul(d[3], mk(-c, sign * c));
    bfly4<C, R>(s, sign);
    bfly4<C, R>(d, sign);
    for (int m = 0; m < 4; ++m) {
      v[2 * m] = s[m];
      v[2 * m + 1] = d[m];
    }
  }
}

// LDS line layout of the compile-time-length FFTs: element i of line l sits at
// l * line_stride(P) + pad(i), with one padding slot after every 8 elements and
// an odd line stride, so that the stride-R writes of the first Stockham pass
// and the line-transposing loads/stores of the x kernels avoid bank conflicts.
// P == 0 (runtime length) keeps the dense layout l * P + i.
__host__ __device__ constexpr int line_stride(int P) { return P == 0 ? 0 : ((P + P / 8) | 1); }
template <int PT>
__device__ inline int lidx(int l, int i, int P) {
  if constexpr (PT == 0)
    return l * P + i;
  else
    return l * line_stride(PT) + i + (i >> 3);
}

template <int P, int RD, int NS, typename R>
__device__ inline void fft_pass_c(const typename V2<R>::T* __restrict__ x,
                                  typename V2<R>::T* __restrict__ y, int nl,
                                  const typename V2<R>::T* __restrict__ tw, R sign) {
  using C = typename V2<R>::T;
  constexpr int NB = P / RD;
  constexpr int TS = P / (NS * RD);
  constexpr int LS = line_stride(P);
  for (int t = threadIdx.x; t < nl * NB; t += blockDim.x) {
    const int l = t / NB;
    const int j = t - l * NB;
    const int k = j % NS;
    const C* xl = x + l * LS;
    C* yl = y + l * LS;
    C v[RD];
#pragma unroll
    for (int r = 0; r < RD; ++r) {
      const int e = j + r * NB;
      v[r] = xl[e + (e >> 3)];
    }
    if (NS > 1) {
#pragma unroll
      for (int r = 1; r < RD; ++r) {
        C w = tw[k * r * TS];
        if (sign > 0) w = conjc(w);
        v[r] = cmul(v[r], w);
      }
    }
    bfly<C, R>(v, RD, sign);
    const int base = (j / NS) * NS * RD + k;
#pragma unroll
    for (int r = 0; r < RD; ++r) {
      const int e = base + r * NS;
      yl[e + (e >> 3)] = v[r];
    }
  }
  __syncthreads();
}

// Radix sequences of the supported compile-time lengths.
template <int P>
struct RadixSeq;
template <> struct RadixSeq<12> { static constexpr int n = 2, r0 = 4, r1 = 3, r2 = 1, r3 = 1; };
template <> struct RadixSeq<24> { static constexpr int n = 2, r0 = 8, r1 = 3, r2 = 1, r3 = 1; };
template <> struct RadixSeq<36> { static constexpr int n = 3, r0 = 4, r1 = 3, r2 = 3, r3 = 1; };
template <> struct RadixSeq<48> { static constexpr int n = 3, r0 = 4, r1 = 4, r2 = 3, r3 = 1; };
template <> struct RadixSeq<72> { static constexpr int n = 3, r0 = 8, r1 = 3, r2 = 3, r3 = 1; };
template <> struct RadixSeq<96> { static constexpr int n = 3, r0 = 8, r1 = 4, r2 = 3, r3 = 1; };
template <> struct RadixSeq<144> { static constexpr int n = 4, r0 = 4, r1 = 4, r2 = 3, r3 = 3; };
template <> struct RadixSeq<192> { static constexpr int n = 3, r0 = 8, r1 = 8, r2 = 3, r3 = 1; };

// Batched FFT of nl lines of length P (line l at a[l*P]); returns the buffer
// holding the result. P == 0 selects the runtime-length lds_fft.
template <typename R, int P>
__device__ typename V2<R>::T* fft_lines(typename V2<R>::T* a, typename V2<R>::T* b, int nl,
                                        const FFTPlan1D& pl, const typename V2<R>::T* tw,
                                        R sign) {
  if constexpr (P == 0) {
    return lds_fft<R>(a, b, nl, pl, tw, sign);
  } else {
    using S = RadixSeq<P>;
    fft_pass_c<P, S::r0, 1, R>(a, b, nl, tw, sign);
    fft_pass_c<P, S::r1, S::r0, R>(b, a, nl, tw, sign);
    if constexpr (S::n == 2) {
      return a;
    } else if constexpr (S::n == 3) {
      fft_pass_c<P, S::r2, S::r0 * S::r1, R>(a, b, nl, tw, sign);
      return b;
    } else {
      fft_pass_c<P, S::r2, S::r0 * S::r1, R>(a, b, nl, tw, sign);
      fft_pass_c<P, S::r3, S::r0 * S::r1 * S::r2, R>(b, a, nl, tw, sign);
      return a;
    }
  }
}

// Supported compile-time lengths (others use the runtime path).
inline bool fft_length_specialised(int P) {
  return P == 12 || P == 24 || P == 36 || P == 48 || P == 72 || P == 96 || P == 144 || P == 192;
}

// ---------------------------------------------------------------------------
// Register-resident DFTs for the four-step line kernels (zline.hip, xline.hip).
// ---------------------------------------------------------------------------
// W_N^a = exp(sign 2 pi i a / N) from the table tw[q] = exp(-2 pi i q / P).
template <int N, int P, typename C, typename R>
__device__ inline C wpow(int a, R sign, const C* tw) {
  const C w = tw[((a % N) * (P / N)) % P];
  return (sign > 0) ? conjc(w) : w;
}

// In-register DFT of length N (natural order in and out):
// X_k = sum_n v_n exp(sign 2 pi i n k / N).
template <int N, int P, typename C, typename R>
__device__ inline void dft_reg(C (&v)[N], R sign, const C* tw) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N == 2 || N == 3 || N == 4 || N == 8) {
    bfly<C, R>(v, N, sign);
  } else {
    constexpr int A = (N % 4 == 0 && N != 12) ? 4 : ((N % 3 == 0) ? 3 : 2);
    constexpr int B = N / A;
    C y[N];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      C t[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n1] = v[B * n1 + n2];
      dft_reg<A, P, C, R>(t, sign, tw);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1)
        y[n2 * A + k1] = (n2 * k1 == 0) ? t[k1] : cmul(t[k1], wpow<N, P, C, R>(n2 * k1, sign, tw));
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      C t[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) t[n2] = y[n2 * A + k1];
      dft_reg<B, P, C, R>(t, sign, tw);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = t[k2];
    }
  }
}

// Lengths P = P1 * P2 with a register line kernel: returns P1 (0 if none).
inline int reg_fft_split(int P) {
  switch (P) {
    case 12: return 4;
    case 18: return 6;
    case 24: return 8;
    case 36: return 6;
    case 48: return 8;
    case 54: return 6;
    case 72: return 8;
    case 96: return 12;
    case 108: return 12;
    case 144: return 16;
    default: return 0;
  }
}

// Expands LAUNCH(P1, P2) for the supported lengths (P must pass reg_fft_split).
#define SP_REG_FFT_DISPATCH(P, LAUNCH) \
  switch (P) {                         \
    case 12: LAUNCH(4, 3); break;      \
    case 18: LAUNCH(6, 3); break;      \
    case 24: LAUNCH(8, 3); break;      \
    case 36: LAUNCH(6, 6); break;      \
    case 48: LAUNCH(8, 6); break;      \
    case 54: LAUNCH(6, 9); break;      \
    case 72: LAUNCH(8, 9); break;      \
    case 96: LAUNCH(12, 8); break;     \
    case 108: LAUNCH(12, 9); break;    \
    default: LAUNCH(16, 9); break;     \
  }

}  // namespace sp

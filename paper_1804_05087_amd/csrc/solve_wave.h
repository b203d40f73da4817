// Wave-parallel building blocks of the per-mode Chebyshev-tau solve.
//
// Every sequential piece of the solve is a first-order linear recurrence along
// one parity chain n = p, p+2, ..., (chain position k, n = p + 2k):
//   quasi-tridiagonal back substitution  p_k = a_k + b_k p_{k+1}
//   forward pass                          P_k = p_k + q_k P_{k-1}
//   Chebyshev derivative                  D_{k} = c_k + D_{k+1}
// and the same shapes in the transposed (adjoint) sweeps. A recurrence
// x_k = a_k + b_k x_{k-1} is the composition of affine maps f_k(x) = a_k + b_k x,
// which is associative, so 32 lanes evaluate it as a segmented scan: each lane
// composes the E consecutive maps it owns (blocked layout, k = lane*E + e),
// a Hillis-Steele scan over the 32 lanes (wave shuffles of width 32) gives every
// lane the composition of all earlier maps, and each lane then replays its own E
// maps. Half a 64-lane wave runs one parity chain, so one wave carries both
// parity classes of a Fourier mode. Arrays live in LDS indexed by n; the
// callers place barriers between steps that exchange data through LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "solve_core.h"

namespace sp {

struct Aff {
  cd a;
  double b;
};

__device__ inline Aff aff_compose(Aff earlier, Aff later) {
  return {later.a + earlier.a * later.b, later.b * earlier.b};
}

__device__ inline Aff aff_shfl_up(Aff m, int d) {
  Aff o;
  o.a.re = __shfl_up(m.a.re, d, 32);
  o.a.im = __shfl_up(m.a.im, d, 32);
  o.b = __shfl_up(m.b, d, 32);
  return o;
}
__device__ inline Aff aff_shfl_down(Aff m, int d) {
  Aff o;
  o.a.re = __shfl_down(m.a.re, d, 32);
  o.a.im = __shfl_down(m.a.im, d, 32);
  o.b = __shfl_down(m.b, d, 32);
  return o;
}

__device__ inline cd sum32(cd v) {
#pragma unroll
  for (int d = 16; d >= 1; d >>= 1) {
    v.re += __shfl_xor(v.re, d, 32);
    v.im += __shfl_xor(v.im, d, 32);
  }
  return v;
}

// x_k = a_k + b_k x_{k-1} for k = 0 .. 32E-1 (x_{-1} = x_init), blocked layout.
template <int E>
__device__ inline void rec_up(const cd (&a)[E], const double (&b)[E], cd x_init, cd (&x)[E],
                              int lane) {
  Aff m{a[0], b[0]};
#pragma unroll
  for (int e = 1; e < E; ++e) m = aff_compose(m, Aff{a[e], b[e]});
#pragma unroll
  for (int d = 1; d < 32; d <<= 1) {
    const Aff o = aff_shfl_up(m, d);
    if (lane >= d) m = aff_compose(o, m);
  }
  Aff ex = aff_shfl_up(m, 1);
  if (lane == 0) ex = Aff{cd(0.0), 1.0};
  cd xv = ex.a + x_init * ex.b;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    xv = a[e] + xv * b[e];
    x[e] = xv;
  }
}

// x_k = a_k + b_k x_{k+1} for k = 32E-1 .. 0 (x_{32E} = x_init), blocked layout.
template <int E>
__device__ inline void rec_down(const cd (&a)[E], const double (&b)[E], cd x_init, cd (&x)[E],
                                int lane) {
  Aff m{a[E - 1], b[E - 1]};
#pragma unroll
  for (int e = E - 2; e >= 0; --e) m = aff_compose(m, Aff{a[e], b[e]});
#pragma unroll
  for (int d = 1; d < 32; d <<= 1) {
    const Aff o = aff_shfl_down(m, d);
    if (lane + d < 32) m = aff_compose(o, m);
  }
  Aff ex = aff_shfl_down(m, 1);
  if (lane == 31) ex = Aff{cd(0.0), 1.0};
  cd xv = ex.a + x_init * ex.b;
#pragma unroll
  for (int e = E - 1; e >= 0; --e) {
    xv = a[e] + xv * b[e];
    x[e] = xv;
  }
}

// Parity-p part of (D^2 - lam) g = r (rows 0..N-2), sum_{n = p mod 2} g_n = beta.
template <int E>
__device__ inline void wsweep(SweepView sw, const double* __restrict__ hw, int N, int p,
                              const cd* __restrict__ r, cd beta, cd* __restrict__ g, int lane) {
  const int n1 = N + 1;
  const int nmax = top_index(N, p);
  const int M = (nmax - p) / 2;
  cd a[E], x[E], P[E];
  double b[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = p + 2 * k;
    if (k >= 1 && k <= M) {
      cd d = r[n - 2] * hw[n];
      if (n <= N - 2) d = d + r[n] * hw[n1 + n];
      if (n + 2 <= N - 2) d = d + r[n + 2] * hw[2 * n1 + n];
      a[e] = d * sw.inv_den[n];
      b[e] = -sw.cc[n] * sw.inv_den[n];
    } else {
      a[e] = cd(0.0);
      b[e] = 1.0;
    }
  }
  rec_down<E>(a, b, cd(0.0), x, lane);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = p + 2 * k;
    if (k >= 1 && k <= M) {
      a[e] = x[e];
      b[e] = sw.q[n];
    } else {
      a[e] = cd(0.0);
      b[e] = 1.0;
    }
  }
  rec_up<E>(a, b, cd(0.0), P, lane);
  cd s(0.0);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    if (k >= 1 && k <= M) s = s + P[e];
  }
  s = sum32(s);
  const cd g0 = (beta - s) * sw.inv_sum[p];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = p + 2 * k;
    if (k == 0)
      g[n] = g0;
    else if (k <= M)
      g[n] = P[e] + g0 * sw.Q[n];
  }
}

// b = D a for the parity-pa entries of a (b: parity 1-pa entries, b_N = 0 if it exists).
template <int E>
__device__ inline void wderiv(int N, int pa, const cd* __restrict__ a, cd* __restrict__ bout,
                              int lane) {
  const int nmax = top_index(N, pa);
  const int K = (nmax - pa) / 2;
  cd c[E], x[E];
  double one[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = pa + 2 * k;
    one[e] = 1.0;
    c[e] = (k <= K && n >= 1) ? a[n] * (2.0 * n) : cd(0.0);
  }
  rec_down<E>(c, one, cd(0.0), x, lane);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = pa + 2 * k;
    if (k <= K && n >= 1) bout[n - 1] = (n == 1) ? x[e] * 0.5 : x[e];
  }
  if (lane == 0 && nmax + 1 <= N) bout[nmax + 1] = cd(0.0);
}

// Transposes (adjoint, beta = 0): rbar = H^T gbar on the parity-p chain.
// db (LDS scratch, indexed by n) receives the intermediate adjoint of the
// right-hand-side combination; the caller must not read it. Two barriers
// are taken inside (all 64 lanes must call together).
template <int E>
__device__ inline void wsweep_T(SweepView sw, const double* __restrict__ hw, int N, int p,
                                const cd* __restrict__ gbar, cd* __restrict__ rbar,
                                cd* __restrict__ db, int lane) {
  const int n1 = N + 1;
  const int nmax = top_index(N, p);
  const int M = (nmax - p) / 2;
  cd s(0.0);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = p + 2 * k;
    if (k == 0)
      s = s + gbar[n];
    else if (k <= M)
      s = s + gbar[n] * sw.Q[n];
  }
  s = sum32(s);
  const cd corr = s * (-sw.inv_sum[p]);
  cd a[E], x[E], y[E];
  double b[E];
  // pbar_k = (gbar_n + corr) + q_{n+2} pbar_{k+1}, k = M..1
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = p + 2 * k;
    if (k >= 1 && k <= M) {
      a[e] = gbar[n] + corr;
      b[e] = (n + 2 <= nmax) ? sw.q[n + 2] : 0.0;
    } else {
      a[e] = cd(0.0);
      b[e] = 1.0;
    }
  }
  rec_down<E>(a, b, cd(0.0), x, lane);
  // y_k = pbar_k - inv_den_{n-2} cc_{n-2} y_{k-1}, k = 1..M ; dbar_k = inv_den_n y_k
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = p + 2 * k;
    if (k >= 1 && k <= M) {
      a[e] = x[e];
      b[e] = (k >= 2) ? -(sw.inv_den[n - 2] * sw.cc[n - 2]) : 0.0;
    } else {
      a[e] = cd(0.0);
      b[e] = 1.0;
    }
  }
  rec_up<E>(a, b, cd(0.0), y, lane);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = p + 2 * k;
    if (k >= 1 && k <= M) db[n] = y[e] * sw.inv_den[n];
  }
  __syncthreads();
  // rbar_m = w1_{m+2} db_{m+2} + w2_m db_m + w3_{m-2} db_{m-2}, m <= N-2
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int m = p + 2 * k;
    if (m <= N) {
      cd v(0.0);
      if (m <= N - 2) {
        if (m + 2 <= nmax) v = v + db[m + 2] * hw[m + 2];
        if (m >= p + 2) v = v + db[m] * hw[n1 + m];
        if (m - 2 >= p + 2) v = v + db[m - 2] * hw[2 * n1 + m - 2];
      }
      rbar[m] = v;
    }
  }
  __syncthreads();
}

// abar = D^T bbar: bbar parity pb entries (n <= N-1), abar parity 1-pb entries:
// abar_m = m * sum_{n < m, n = pb mod 2} (2/c_n) bbar_n. S (LDS scratch by n)
// receives the running sums. One barrier inside.
template <int E>
__device__ inline void wderiv_T(int N, int pb, const cd* __restrict__ bbar, cd* __restrict__ abar,
                                cd* __restrict__ S, int lane) {
  const int nmaxb = top_index(N, pb);
  const int Kb = (nmaxb - pb) / 2;
  cd c[E], x[E];
  double one[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = pb + 2 * k;
    one[e] = 1.0;
    c[e] = (k <= Kb && n <= N - 1) ? bbar[n] * ((n == 0) ? 1.0 : 2.0) : cd(0.0);
  }
  rec_up<E>(c, one, cd(0.0), x, lane);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int n = pb + 2 * k;
    if (k <= Kb) S[n] = x[e];
  }
  __syncthreads();
  const int pa = 1 - pb;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = lane * E + e;
    const int m = pa + 2 * k;
    if (m <= N) abar[m] = (m >= 1) ? S[m - 1] * (double)m : cd(0.0);
  }
}

}  // namespace sp

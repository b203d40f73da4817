// Per-mode Chebyshev-tau solve: building blocks shared by the host precompute
// (real arithmetic) and the device kernel (complex arithmetic).
//
// The implicit BEFE solve of one Fourier mode (k_x, k_z), k = |(k_x, k_z)| > 0,
// in the form (multiplied by Re, P = Re p, F = Re g, lam = k^2 + Re/dt)
//
//   (D^2 - lam) u - grad P = -F  on T_0..T_{N-2},  u = 0 at y = +-1,
//   i k_x u + D v + i k_z w = 0  on T_0..T_N,
//
// is rotated to (u_par, u_perp) = ((k_x u + k_z w)/k, (k_z u - k_x w)/k):
// u_perp solves a Dirichlet Helmholtz problem; continuity gives
// u_par = i D v / k exactly, and (v, P) solve
//
//   (D^2 - k^2) P = div F - b D T_m            on T_0..T_{N-2}, P(+-1) = delta
//   (D^2 - lam) v = D P - F_v                  on T_0..T_{N-2}, v(+-1) = 0
//
// where the tau coefficient b of the v equation (m in {N-1, N}) and the
// Dirichlet value delta of P are fixed by D v(+-1) = 0 and by the definition
// of b; both enter linearly, so a particular solution plus two precomputed
// influence solutions per parity class reproduce the coupled system exactly
// (the influence-matrix technique with tau correction, paper Sec. 3.2).
// Everything splits by the parity of the Chebyshev index: class pv holds v of
// parity pv and P, u_par, u_perp of the other parity.
//
// Each Dirichlet problem (D^2 - lam) g = r (rows 0..N-2), sum over n of parity p
// of g_n = beta, is solved in the quasi-tridiagonal form obtained by expressing
// g_n through the coefficients of g'' (Chebyshev recurrence), n = 2..N:
//   -c_{n-2} lam/(4n(n-1)) g_{n-2} + (1 + e_{n+2} lam/(2(n^2-1))) g_n
//        - e_{n+4} lam/(4n(n+1)) g_{n+2}
//   = c_{n-2} r_{n-2}/(4n(n-1)) - e_{n+2} r_n/(2(n^2-1)) + e_{n+4} r_{n+2}/(4n(n+1)),
// c_0 = 2, c_j = 1 otherwise, e_j = 1 if j <= N else 0. A backward sweep
// eliminates the upper band, the wall row fixes the first unknown, and a
// parallel pass recovers the rest.
#pragma once

#include <hip/hip_runtime.h>

namespace sp {

struct cd {
  double re, im;
  __host__ __device__ cd() : re(0.0), im(0.0) {}
  __host__ __device__ cd(double r) : re(r), im(0.0) {}
  __host__ __device__ cd(double r, double i) : re(r), im(i) {}
};
__host__ __device__ inline cd operator+(cd a, cd b) { return cd(a.re + b.re, a.im + b.im); }
__host__ __device__ inline cd operator-(cd a, cd b) { return cd(a.re - b.re, a.im - b.im); }
__host__ __device__ inline cd operator-(cd a) { return cd(-a.re, -a.im); }
__host__ __device__ inline cd operator*(cd a, double s) { return cd(a.re * s, a.im * s); }
__host__ __device__ inline cd operator*(double s, cd a) { return cd(a.re * s, a.im * s); }
__host__ __device__ inline cd mul_i(cd a) { return cd(-a.im, a.re); }  // i * a

// Offsets inside a sweep block of n1 = N + 1: inv_den, cc, q, Q, inv_sum_q[2].
struct SweepView {
  const double* inv_den;
  const double* cc;
  const double* q;
  const double* Q;
  const double* inv_sum;
  __host__ __device__ SweepView(const double* base, int n1)
      : inv_den(base), cc(base + n1), q(base + 2 * n1), Q(base + 3 * n1), inv_sum(base + 4 * n1) {}
};

// Right-hand-side weights hw = [w1 | w2 | w3], each of length n1.
__host__ __device__ inline int top_index(int N, int p) { return ((N - p) % 2 == 0) ? N : N - 1; }

// Solves the parity-p part of (D^2 - lam) g = r, rows 0..N-2, sum_{n = p mod 2} g_n = beta.
// r entries above N-2 are ignored. work: scratch of length n1 (parity-p entries used).
template <typename T>
__host__ __device__ inline void sweep_solve(SweepView sw, const double* hw, int N, int p,
                                            const T* r, T beta, T* g, T* work) {
  const int n1 = N + 1;
  const double* w1 = hw;
  const double* w2 = hw + n1;
  const double* w3 = hw + 2 * n1;
  const int nmax = top_index(N, p);
  T pnext = T(0.0);
  for (int n = nmax; n >= p + 2; n -= 2) {
    T d = r[n - 2] * w1[n];
    if (n <= N - 2) d = d + r[n] * w2[n];
    if (n + 2 <= N - 2) d = d + r[n + 2] * w3[n];
    T pn = (d - pnext * sw.cc[n]) * sw.inv_den[n];
    work[n] = pn;
    pnext = pn;
  }
  T prev = T(0.0);
  T sum = T(0.0);
  for (int n = p + 2; n <= nmax; n += 2) {
    T P = work[n] + prev * sw.q[n];
    work[n] = P;
    sum = sum + P;
    prev = P;
  }
  T g0 = (beta - sum) * sw.inv_sum[p];
  g[p] = g0;
  for (int n = p + 2; n <= nmax; n += 2) g[n] = work[n] + g0 * sw.Q[n];
}

// b = D a for the parity-pa entries of a (b gets parity 1 - pa, entries n <= N-1).
template <typename T>
__host__ __device__ inline void deriv_parity(int N, int pa, const T* a, T* b) {
  const int nmax = top_index(N, pa);
  T bnext = T(0.0);  // b_{n+1}
  for (int n = nmax; n >= 1; n -= 2) {
    T bn = bnext + a[n] * (2.0 * n);
    b[n - 1] = bn;
    bnext = bn;
  }
  if (pa == 1) b[0] = b[0] * 0.5;
  if (nmax + 1 <= N) b[nmax + 1] = T(0.0);
}

// Precomputes the sweep block of the operator (D^2 - lam) for both parities.
inline void sweep_factor(int N, double lam, double* blk) {
  const int n1 = N + 1;
  double* inv_den = blk;
  double* cc = blk + n1;
  double* q = blk + 2 * n1;
  double* Q = blk + 3 * n1;
  double* inv_sum = blk + 4 * n1;
  for (int i = 0; i < 4 * n1 + 2; ++i) blk[i] = 0.0;
  for (int p = 0; p < 2; ++p) {
    const int nmax = top_index(N, p);
    double qnext = 0.0;
    for (int n = nmax; n >= p + 2; n -= 2) {
      const double cnm2 = (n - 2 == 0) ? 2.0 : 1.0;
      const double a = -cnm2 * lam / (4.0 * n * (n - 1));
      const double b = 1.0 + ((n + 2 <= N) ? lam / (2.0 * (n * (double)n - 1.0)) : 0.0);
      const double c = (n + 4 <= N) ? -lam / (4.0 * n * (n + 1)) : 0.0;
      const double den = b + c * qnext;
      q[n] = -a / den;
      inv_den[n] = 1.0 / den;
      cc[n] = c;
      qnext = q[n];
    }
    Q[p] = 1.0;
    double sum = 1.0;
    for (int n = p + 2; n <= nmax; n += 2) {
      Q[n] = q[n] * Q[n - 2];
      sum += Q[n];
    }
    inv_sum[p] = 1.0 / sum;
  }
}

// Right-hand-side weights of the quasi-tridiagonal form (length 3 n1).
inline void rhs_weights(int N, double* hw) {
  const int n1 = N + 1;
  for (int i = 0; i < 3 * n1; ++i) hw[i] = 0.0;
  for (int n = 2; n <= N; ++n) {
    const double cnm2 = (n - 2 == 0) ? 2.0 : 1.0;
    hw[n] = cnm2 / (4.0 * n * (n - 1));
    hw[n1 + n] = (n + 2 <= N) ? -1.0 / (2.0 * (n * (double)n - 1.0)) : 0.0;
    hw[2 * n1 + n] = (n + 4 <= N) ? 1.0 / (4.0 * n * (n + 1)) : 0.0;
  }
}

}  // namespace sp

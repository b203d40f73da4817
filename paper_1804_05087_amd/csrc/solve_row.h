// Row-parallel building blocks of the per-mode Chebyshev-tau solve.
//
// Every sequential piece of the solve is a first-order linear recurrence along
// one parity chain n = p, p+2, ..., (chain position k, n = p + 2k):
//   quasi-tridiagonal back substitution  p_k = a_k + b_k p_{k+1}
//   forward pass                          P_k = p_k + q_k P_{k-1}
//   Chebyshev derivative                  D_k = c_k + D_{k+1}
// and the same shapes in the transposed (adjoint) sweeps. x_k = a_k + b_k x_{k-1}
// is the composition of the affine maps f_k(x) = a_k + b_k x, which is
// associative, so one 16-lane row of the wave evaluates a chain as a segmented
// scan: each lane composes the E consecutive maps it owns (k = l E + e, l = lane
// within the row), a Hillis-Steele scan over the row combines them, and each
// lane replays its own maps. The scan steps move data with DPP row shifts
// (row_shr / row_shl: from the lane d below / above within the row; lanes whose
// source lies outside the row receive the identity map), so a chain never
// leaves the vector registers. The four rows of a wave run four chains in one
// instruction stream; every argument that selects a chain (parity, arrays,
// factors) may differ from row to row. Arrays live in LDS indexed by n; the
// callers place barriers between steps that exchange data through LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "solve_core.h"

namespace sp {

struct Aff {
  cd a;
  double b;
};

// apply `earlier`, then `later`
__device__ inline Aff aff_compose(Aff earlier, Aff later) {
  return {later.a + earlier.a * later.b, later.b * earlier.b};
}

constexpr int kDppRowShl = 0x100;  // lane l <- lane l + n (same row)
constexpr int kDppRowShr = 0x110;  // lane l <- lane l - n (same row)
constexpr int kDppRowRor = 0x120;  // lane l <- lane (l - n) mod 16

// One DPP move of a double; lanes without a source in the row keep `old`.
template <int CTRL>
__device__ inline double dpp_mov(double v, double old) {
  const long long vi = __double_as_longlong(v);
  const long long oi = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)oi, (int)vi, CTRL, 0xF, 0xF, false);
  const int hi =
      __builtin_amdgcn_update_dpp((int)(oi >> 32), (int)(vi >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

template <int CTRL>
__device__ inline Aff aff_dpp(Aff m) {
  return {cd(dpp_mov<CTRL>(m.a.re, 0.0), dpp_mov<CTRL>(m.a.im, 0.0)), dpp_mov<CTRL>(m.b, 1.0)};
}

template <int CTRL>
__device__ inline cd cd_dpp(cd v) {
  return cd(dpp_mov<CTRL>(v.re, 0.0), dpp_mov<CTRL>(v.im, 0.0));
}

// Sum over the 16 lanes of the row, returned in every lane of the row.
__device__ inline cd row_sum(cd v) {
  v = v + cd_dpp<kDppRowRor | 8>(v);
  v = v + cd_dpp<kDppRowRor | 4>(v);
  v = v + cd_dpp<kDppRowRor | 2>(v);
  v = v + cd_dpp<kDppRowRor | 1>(v);
  return v;
}

// x_k = a_k + b_k x_{k-1} for k = 0 .. 16E-1 (x_{-1} = x_init), blocked layout.
template <int E>
__device__ inline void rec_up(const cd (&a)[E], const double (&b)[E], cd x_init, cd (&x)[E]) {
  Aff m{a[0], b[0]};
#pragma unroll
  for (int e = 1; e < E; ++e) m = aff_compose(m, Aff{a[e], b[e]});
  m = aff_compose(aff_dpp<kDppRowShr | 1>(m), m);
  m = aff_compose(aff_dpp<kDppRowShr | 2>(m), m);
  m = aff_compose(aff_dpp<kDppRowShr | 4>(m), m);
  m = aff_compose(aff_dpp<kDppRowShr | 8>(m), m);
  const Aff ex = aff_dpp<kDppRowShr | 1>(m);  // maps of all lower lanes (identity in lane 0)
  cd xv = ex.a + x_init * ex.b;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    xv = a[e] + xv * b[e];
    x[e] = xv;
  }
}

// x_k = a_k + b_k x_{k+1} for k = 16E-1 .. 0 (x_{16E} = x_init), blocked layout.
template <int E>
__device__ inline void rec_down(const cd (&a)[E], const double (&b)[E], cd x_init, cd (&x)[E]) {
  Aff m{a[E - 1], b[E - 1]};
#pragma unroll
  for (int e = E - 2; e >= 0; --e) m = aff_compose(m, Aff{a[e], b[e]});
  m = aff_compose(aff_dpp<kDppRowShl | 1>(m), m);
  m = aff_compose(aff_dpp<kDppRowShl | 2>(m), m);
  m = aff_compose(aff_dpp<kDppRowShl | 4>(m), m);
  m = aff_compose(aff_dpp<kDppRowShl | 8>(m), m);
  const Aff ex = aff_dpp<kDppRowShl | 1>(m);  // maps of all higher lanes (identity in lane 15)
  cd xv = ex.a + x_init * ex.b;
#pragma unroll
  for (int e = E - 1; e >= 0; --e) {
    xv = a[e] + xv * b[e];
    x[e] = xv;
  }
}

// The element loads below use indexes clamped into the chain and 0/1 masks
// applied to the loaded values instead of per-element branches: a load under
// a per-lane condition is compiled into its own branch followed by a wait for
// it, which serialises the LDS round trips.
__device__ inline double mask(bool c) { return c ? 1.0 : 0.0; }

// Sweep data of one operator (D^2 - lam) in a mode record: inv_den, Q and
// inv_sum stored, the band and pass factors formed from lam and the
// right-hand-side weights w1 = hw, w3 = hw + 2 n1 of the quasi-tridiagonal
// form: cc_n = -lam w3_n, q_n = lam w1_n inv_den_n (solve_core.h).
struct SweepRec {
  const double* inv_den;
  const double* Q;
  const double* inv_sum;
  double lam;
  __device__ SweepRec(const double* base, int n1, double lam_)
      : inv_den(base), Q(base + n1), inv_sum(base + 2 * n1), lam(lam_) {}
};

// Parity-p part of (D^2 - lam) g = r (rows 0..N-2), sum_{n = p mod 2} g_n = beta.
template <int E>
__device__ inline void wsweep(SweepRec sw, const double* __restrict__ hw, int N, int p,
                              const cd* r, cd beta, cd* g, int l) {
  const int n1 = N + 1;
  const int nmax = top_index(N, p);
  const int M = (nmax - p) / 2;
  const double inv_sum = sw.inv_sum[p];
  cd a[E], x[E], P[E];
  double b[E], qv[E], Qv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int n = p + 2 * k;
    const double act = mask(k >= 1 && k <= M);
    const int nc = (k < 1) ? p + 2 : (k > M ? nmax : n);  // a valid chain element >= 2
    const cd rm = r[nc - 2];
    const cd r0 = r[nc];
    const cd rp = r[nc + 2 <= nmax ? nc + 2 : nmax];  // same parity: written by the caller
    const double w1 = hw[nc];
    const double w2 = hw[n1 + nc] * mask(nc <= N - 2);
    const double w3 = hw[2 * n1 + nc] * mask(nc + 2 <= N - 2);
    const double id = sw.inv_den[nc];
    qv[e] = sw.lam * w1 * id * act;  // q = lam w1 / den
    Qv[e] = sw.Q[nc];
    a[e] = (rm * w1 + r0 * w2 + rp * w3) * (id * act);
    b[e] = fma(sw.lam * w3 * id, act, 1.0 - act);  // -cc / den = lam w3 / den on the chain, 1 elsewhere
  }
  rec_down<E>(a, b, cd(0.0), x);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const double act = mask(k >= 1 && k <= M);
    a[e] = x[e] * act;
    b[e] = qv[e] + (1.0 - act);  // q on the chain, 1 elsewhere
  }
  rec_up<E>(a, b, cd(0.0), P);
  cd s(0.0);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    s = s + P[e] * mask(k >= 1 && k <= M);
  }
  s = row_sum(s);
  const cd g0 = (beta - s) * inv_sum;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int n = p + 2 * k;
    if (k == 0)
      g[n] = g0;
    else if (k <= M)
      g[n] = P[e] + g0 * Qv[e];
  }
}

// Stores its argument (the plain derivative).
struct StoreDeriv {
  __device__ cd operator()(int, cd v) const { return v; }
};

// Uses the loaded entry as it is.
struct LoadDeriv {
  __device__ cd operator()(int, cd v, bool) const { return v; }
};

// b = D a for the parity-pa entries of a (b: parity 1-pa entries, b_N = 0 if it exists);
// bout[m] receives post(m, b_m), so that an element-wise step on b is taken where
// each entry is stored, and entry a_n enters as pre(n, a_n, own), own telling the
// one lane that owns n (the lane of chain position (n - pa) / 2, as in SP_ROW_PAR),
// so that an element-wise step on a is taken where each entry is loaded.
template <int E, class Post = StoreDeriv, class Pre = LoadDeriv>
__device__ inline void wderiv(int N, int pa, const cd* a, cd* bout, int l, Post post = Post(),
                              Pre pre = Pre()) {
  const int nmax = top_index(N, pa);
  const int K = (nmax - pa) / 2;
  cd c[E], x[E];
  double one[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int n = pa + 2 * k;
    one[e] = 1.0;
    const int nc = (k <= K) ? n : nmax;
    c[e] = pre(nc, a[nc], k <= K) * ((2.0 * n) * mask(k <= K && n >= 1));
  }
  rec_down<E>(c, one, cd(0.0), x);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int n = pa + 2 * k;
    if (k <= K && n >= 1) bout[n - 1] = post(n - 1, (n == 1) ? x[e] * 0.5 : x[e]);
  }
  if (l == 0 && nmax + 1 <= N) bout[nmax + 1] = post(nmax + 1, cd(0.0));
}

// Transposes (adjoint, beta = 0): rbar = H^T gbar on the parity-p chain.
// db (LDS scratch indexed by n, distinct per row) receives the intermediate
// adjoint of the right-hand-side combination. Two barriers are taken inside
// (every lane of the block must call together).
template <int E>
__device__ inline void wsweep_T(SweepRec sw, const double* __restrict__ hw, int N, int p,
                                const cd* gbar, cd* rbar, cd* db, int l) {
  const int n1 = N + 1;
  const int nmax = top_index(N, p);
  const int M = (nmax - p) / 2;
  const double inv_sum = sw.inv_sum[p];
  cd gv[E];
  double Qv[E], q2[E], id[E], cm[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int n = p + 2 * k;
    const int nc = (k <= M) ? n : nmax;
    const int nc2 = (k >= 2 && k <= M) ? n - 2 : p;
    const int np2 = nc + 2 <= nmax ? nc + 2 : nmax;
    gv[e] = gbar[nc] * mask(k <= M);
    Qv[e] = (k == 0) ? 1.0 : sw.Q[nc];
    q2[e] = sw.lam * hw[np2] * sw.inv_den[np2] * mask(n + 2 <= nmax);  // q_{n+2}
    id[e] = sw.inv_den[nc];
    cm[e] = -sw.lam * hw[2 * n1 + nc2] * sw.inv_den[nc2];  // inv_den cc at n - 2
  }
  cd s(0.0);
#pragma unroll
  for (int e = 0; e < E; ++e) s = s + gv[e] * Qv[e];
  s = row_sum(s);
  const cd corr = s * (-inv_sum);
  cd a[E], x[E], y[E];
  double b[E];
  // pbar_k = (gbar_n + corr) + q_{n+2} pbar_{k+1}, k = M..1
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const double act = mask(k >= 1 && k <= M);
    a[e] = (gv[e] + corr) * act;
    b[e] = q2[e] * act + (1.0 - act);
  }
  rec_down<E>(a, b, cd(0.0), x);
  // y_k = pbar_k - inv_den_{n-2} cc_{n-2} y_{k-1}, k = 1..M ; dbar_k = inv_den_n y_k
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const double act = mask(k >= 1 && k <= M);
    a[e] = x[e] * act;
    b[e] = -cm[e] * mask(k >= 2 && k <= M) + (1.0 - act);
  }
  rec_up<E>(a, b, cd(0.0), y);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int n = p + 2 * k;
    if (k >= 1 && k <= M) db[n] = y[e] * id[e];
  }
  __syncthreads();
  // rbar_m = w1_{m+2} db_{m+2} + w2_m db_m + w3_{m-2} db_{m-2}, m <= N-2
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int m = p + 2 * k;
    // db holds entries k = 1..M only (M >= 1): every index below stays among them
    const int mc = (k >= 1 && k <= M) ? m : p + 2;
    const int mp = m + 2 <= nmax ? m + 2 : nmax;
    const int mm = m - 2 >= p + 2 && k <= M ? m - 2 : p + 2;
    const double f = mask(m <= N - 2);
    const cd v = db[mp] * (hw[mp] * f * mask(m + 2 <= nmax)) +
                 db[mc] * (hw[n1 + mc] * f * mask(m >= p + 2)) +
                 db[mm] * (hw[2 * n1 + mm] * f * mask(m - 2 >= p + 2));
    if (m <= N) rbar[m] = v;
  }
  __syncthreads();
}

// abar = D^T bbar: bbar parity pb entries (n <= N-1), abar parity 1-pb entries:
// abar_m = m * sum_{n < m, n = pb mod 2} (2/c_n) bbar_n. S (LDS scratch by n,
// distinct per row) receives the running sums. One barrier inside.
template <int E>
__device__ inline void wderiv_T(int N, int pb, const cd* bbar, cd* abar, cd* S, int l) {
  const int nmaxb = top_index(N, pb);
  const int Kb = (nmaxb - pb) / 2;
  cd c[E], x[E];
  double one[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int n = pb + 2 * k;
    one[e] = 1.0;
    const int nc = (k <= Kb) ? n : nmaxb;
    c[e] = bbar[nc] * (((n == 0) ? 1.0 : 2.0) * mask(k <= Kb && n <= N - 1));
  }
  rec_up<E>(c, one, cd(0.0), x);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int n = pb + 2 * k;
    if (k <= Kb) S[n] = x[e];
  }
  __syncthreads();
  const int pa = 1 - pb;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = l * E + e;
    const int m = pa + 2 * k;
    const int mc = (m <= N) ? m : N - ((N - pa) % 2);
    const cd v = S[mc >= 1 ? mc - 1 : pb] * ((double)m * mask(m >= 1));  // S holds parity pb
    if (m <= N) abar[m] = v;
  }
}

}  // namespace sp

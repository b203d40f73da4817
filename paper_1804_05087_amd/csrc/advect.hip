// The BEFE step with the laminar advection moved into the implicit operator
// (paper Sec. 6, the proposed remedy for the Krylov counts at high Re):
//
//   (I - dt (L + M)) Phi~(U) = U + dt (N(U) - M U),
//   M u = -( i k_x y u + v, i k_x y v, i k_x y w )    per Fourier mode,
//
// the linearisation of the advection about U_lam = y e_x in convective form.
// Multiplication by y couples neighbouring Chebyshev coefficients of both
// parities, so the per-mode system no longer splits into the parity chains of
// the Stokes solve. The plan therefore builds, once per (Re, dt), each mode's
// dense solution operator S~_k (the tau system's map from the 3 (N-1) used
// right-hand-side coefficients to the 3 (N+1) velocity coefficients) on the
// host, by LU with partial pivoting and iterative refinement with
// extended-precision residuals, and the step applies it as a per-mode complex
// matrix-vector product. The mean mode (k_x = 0, v = 0) is unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "device_common.h"
#include "sp_internal.h"

namespace sp {

bool adv_mode_operator(int N, double kx, double kz, double re, double inv_dt,
                       std::complex<double>* S);

namespace {

using cplx = std::complex<double>;
using cplxl = std::complex<long double>;

// Dense tau system of one mode (k != 0): unknowns u_0..u_N, v_0..v_N,
// w_0..w_N, p_0..p_N; rows: x-, y-, z-momentum on T_0..T_{N-2}, the six
// no-slip rows, continuity on T_0..T_N. A is row-major (4 n1)^2.
void adv_mode_matrix(int N, double kx, double kz, double re, double inv_dt,
                     std::vector<cplx>& A) {
  const int n1 = N + 1, n4 = 4 * n1;
  A.assign((size_t)n4 * n4, cplx(0.0, 0.0));
  // D (coefficients of d/dy), D2 = D D, both exact small integers
  std::vector<double> D((size_t)n1 * n1, 0.0), D2((size_t)n1 * n1, 0.0);
  for (int n = 0; n < n1; ++n)
    for (int m = n + 1; m < n1; ++m)
      if ((m + n) % 2 == 1) D[(size_t)n * n1 + m] = (n == 0 ? 1.0 : 2.0) * m;
  for (int n = 0; n < n1; ++n)
    for (int m = 0; m < n1; ++m) {
      double s = 0.0;
      for (int q = 0; q < n1; ++q) s += D[(size_t)n * n1 + q] * D[(size_t)q * n1 + m];
      D2[(size_t)n * n1 + m] = s;
    }
  const double k2 = kx * kx + kz * kz;
  const double diag = k2 / re + inv_dt;
  auto at = [&](int r, int c) -> cplx& { return A[(size_t)r * n4 + c]; };
  const int U = 0, V = n1, W = 2 * n1, P = 3 * n1;
  const cplx ikx(0.0, kx), ikz(0.0, kz);
  // momentum rows: (D2/Re - (k^2/Re + 1/dt)) - i kx Y on the component's block
  for (int comp = 0; comp < 3; ++comp) {
    const int off = comp * n1;
    for (int n = 0; n <= N - 2; ++n) {
      const int r = comp * (N - 1) + n;
      for (int m = 0; m < n1; ++m) at(r, off + m) = cplx(D2[(size_t)n * n1 + m] / re, 0.0);
      at(r, off + n) -= diag;
      // -(i kx y): (y a)_n = a_1/2 (n = 0); a_0 + a_2/2 (n = 1); (a_{n-1} + a_{n+1})/2
      if (n == 0) {
        at(r, off + 1) -= 0.5 * ikx;
      } else {
        at(r, off + n - 1) -= (n == 1 ? 1.0 : 0.5) * ikx;
        at(r, off + n + 1) -= 0.5 * ikx;
      }
      if (comp == 0) {
        at(r, V + n) -= 1.0;  // -(u . grad) U_lam = -v e_x
        at(r, P + n) = -ikx;
      } else if (comp == 1) {
        for (int m = 0; m < n1; ++m) at(r, P + m) = cplx(-D[(size_t)n * n1 + m], 0.0);
      } else {
        at(r, P + n) = -ikz;
      }
    }
  }
  int r = 3 * (N - 1);
  for (int off : {U, V, W}) {  // u(1) = 0, u(-1) = 0
    for (int m = 0; m < n1; ++m) at(r, off + m) = 1.0;
    ++r;
    for (int m = 0; m < n1; ++m) at(r, off + m) = (m % 2) ? -1.0 : 1.0;
    ++r;
  }
  for (int n = 0; n < n1; ++n, ++r) {  // i kx u + D v + i kz w = 0, every coefficient
    at(r, U + n) = ikx;
    for (int m = 0; m < n1; ++m) at(r, V + m) = cplx(D[(size_t)n * n1 + m], 0.0);
    at(r, W + n) = ikz;
  }
}

// In-place LU with partial pivoting (row-major n x n). Returns false if
// singular.
bool lu_factor(std::vector<cplx>& LU, int n, std::vector<int>& piv) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(LU[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      const double v = std::abs(LU[(size_t)i * n + k]);
      if (v > best) best = v, p = i;
    }
    if (!(best > 0.0)) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(LU[(size_t)k * n + j], LU[(size_t)p * n + j]);
    const cplx inv = 1.0 / LU[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      cplx& lik = LU[(size_t)i * n + k];
      if (lik == cplx(0.0, 0.0)) continue;
      lik *= inv;
      const double fr = lik.real(), fi = lik.imag();
      double* ri = reinterpret_cast<double*>(&LU[(size_t)i * n]);
      const double* rk = reinterpret_cast<const double*>(&LU[(size_t)k * n]);
      for (int j = k + 1; j < n; ++j) {
        const double ar = rk[2 * j], ai = rk[2 * j + 1];
        ri[2 * j] -= fr * ar - fi * ai;
        ri[2 * j + 1] -= fr * ai + fi * ar;
      }
    }
  }
  return true;
}

}  // namespace

namespace {

// Sparse rows of a row-major n x n complex matrix restricted to columns
// [lo(i), hi(i)) of row i: column indices and values.
struct SparseRows {
  std::vector<int> start, col;
  std::vector<double> re, im;
  template <typename Lo, typename Hi>
  void build(const std::vector<cplx>& M, int n, Lo lo, Hi hi) {
    start.assign(n + 1, 0);
    col.clear();
    re.clear();
    im.clear();
    for (int i = 0; i < n; ++i) {
      for (int j = lo(i); j < hi(i); ++j) {
        const cplx v = M[(size_t)i * n + j];
        if (v == cplx(0.0, 0.0)) continue;
        col.push_back(j);
        re.push_back(v.real());
        im.push_back(v.imag());
      }
      start[i + 1] = (int)col.size();
    }
  }
};

// X <- (LU)^{-1} P X for the C right-hand sides held as rows of X (row-major
// n x C, real and imaginary parts apart so that the column loops vectorise).
void lu_solve_multi(const SparseRows& L, const SparseRows& U, const std::vector<cplx>& diag_inv,
                    const std::vector<int>& piv, int n, int C, double* Xr, double* Xi) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) {
      std::swap_ranges(Xr + (size_t)k * C, Xr + (size_t)(k + 1) * C, Xr + (size_t)piv[k] * C);
      std::swap_ranges(Xi + (size_t)k * C, Xi + (size_t)(k + 1) * C, Xi + (size_t)piv[k] * C);
    }
  for (int i = 1; i < n; ++i) {
    double* xr = Xr + (size_t)i * C;
    double* xi = Xi + (size_t)i * C;
    for (int q = L.start[i]; q < L.start[i + 1]; ++q) {
      const double lr = L.re[q], li = L.im[q];
      const double* yr = Xr + (size_t)L.col[q] * C;
      const double* yi = Xi + (size_t)L.col[q] * C;
      for (int c = 0; c < C; ++c) {
        xr[c] -= lr * yr[c] - li * yi[c];
        xi[c] -= lr * yi[c] + li * yr[c];
      }
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double* xr = Xr + (size_t)i * C;
    double* xi = Xi + (size_t)i * C;
    for (int q = U.start[i]; q < U.start[i + 1]; ++q) {
      const double ur = U.re[q], ui = U.im[q];
      const double* yr = Xr + (size_t)U.col[q] * C;
      const double* yi = Xi + (size_t)U.col[q] * C;
      for (int c = 0; c < C; ++c) {
        xr[c] -= ur * yr[c] - ui * yi[c];
        xi[c] -= ur * yi[c] + ui * yr[c];
      }
    }
    const double dr = diag_inv[i].real(), di = diag_inv[i].imag();
    for (int c = 0; c < C; ++c) {
      const double a = xr[c], b = xi[c];
      xr[c] = a * dr - b * di;
      xi[c] = a * di + b * dr;
    }
  }
}

}  // namespace

// S~ of one mode, column-major: S[col * 3 n1 + row], col < 3 (N-1) the used
// right-hand-side coefficient (component col / (N-1), index col % (N-1)).
// The tau system reads (operator) phi = -g, so column col solves A x = -e_col.
// All columns are solved together, and the solution is refined twice with
// residuals accumulated in long double over the non-zeros of A (about a tenth
// of its entries).
bool adv_mode_operator(int N, double kx, double kz, double re, double inv_dt, cplx* S) {
  const int n1 = N + 1, n4 = 4 * n1, R = 3 * n1, C = 3 * (N - 1);
  std::vector<cplx> A, LU;
  adv_mode_matrix(N, kx, kz, re, inv_dt, A);
  LU = A;
  std::vector<int> piv;
  if (!lu_factor(LU, n4, piv)) return false;
  SparseRows Ar, L, U;
  Ar.build(A, n4, [](int) { return 0; }, [n4](int) { return n4; });
  L.build(LU, n4, [](int) { return 0; }, [](int i) { return i; });
  U.build(LU, n4, [](int i) { return i + 1; }, [n4](int) { return n4; });
  std::vector<cplx> dinv(n4);
  for (int i = 0; i < n4; ++i) dinv[i] = 1.0 / LU[(size_t)i * n4 + i];
  std::vector<double> Xr((size_t)n4 * C, 0.0), Xi((size_t)n4 * C, 0.0);
  std::vector<double> Rr((size_t)n4 * C), Ri((size_t)n4 * C);
  for (int col = 0; col < C; ++col) Xr[(size_t)col * C + col] = -1.0;
  lu_solve_multi(L, U, dinv, piv, n4, C, Xr.data(), Xi.data());
  std::vector<long double> sr(C), si(C);
  for (int it = 0; it < 2; ++it) {
    for (int i = 0; i < n4; ++i) {  // residual -e - A X, row i for every column
      std::fill(sr.begin(), sr.end(), 0.0L);
      std::fill(si.begin(), si.end(), 0.0L);
      if (i < C) sr[i] = -1.0L;
      for (int q = Ar.start[i]; q < Ar.start[i + 1]; ++q) {
        const long double ar = Ar.re[q], ai = Ar.im[q];
        const double* xr = &Xr[(size_t)Ar.col[q] * C];
        const double* xi = &Xi[(size_t)Ar.col[q] * C];
        for (int c = 0; c < C; ++c) {
          sr[c] -= ar * xr[c] - ai * xi[c];
          si[c] -= ar * xi[c] + ai * xr[c];
        }
      }
      for (int c = 0; c < C; ++c) {
        Rr[(size_t)i * C + c] = (double)sr[c];
        Ri[(size_t)i * C + c] = (double)si[c];
      }
    }
    lu_solve_multi(L, U, dinv, piv, n4, C, Rr.data(), Ri.data());
    for (size_t e = 0; e < Xr.size(); ++e) {
      Xr[e] += Rr[e];
      Xi[e] += Ri[e];
    }
  }
  for (int col = 0; col < C; ++col)
    for (int i = 0; i < R; ++i)
      S[(size_t)col * R + i] = cplx(Xr[(size_t)i * C + col], Xi[(size_t)i * C + col]);
  return true;
}

namespace {

// out_k = S~_k (g_k + i k_x Y x_k + (x_v, 0, 0)) on the used coefficients,
// one block per mode; the mean mode and the Nyquist modes are skipped (their
// output comes from the Stokes solve).
__global__ void __launch_bounds__(256)
    k_adv_apply(const double2* __restrict__ g, const double2* __restrict__ x,
                const double2* __restrict__ S, double2* __restrict__ out, int nx, int ny,
                int nzh, double alpha) {
  extern __shared__ unsigned char smem_raw[];
  double2* gl = reinterpret_cast<double2*>(smem_raw);
  const int mode = blockIdx.x;
  const int i = mode / nzh;
  const int j = mode - i * nzh;
  if ((i == 0 && j == 0) || i == nx / 2 || j == nzh - 1) return;  // block-uniform
  const int N = ny - 1;
  const int C = 3 * (N - 1), R = 3 * ny;
  const size_t cs = (size_t)nx * nzh * ny;
  const size_t mo = (size_t)mode * ny;
  const double kx = alpha * (double)(i < nx / 2 ? i : i - nx);
  for (int t = threadIdx.x; t < C; t += blockDim.x) {
    const int c = t / (N - 1);
    const int n = t - c * (N - 1);
    const double2* a = x + c * cs + mo;
    double2 y;  // (y a)_n
    if (n == 0) {
      y = make_double2(0.5 * a[1].x, 0.5 * a[1].y);
    } else {
      const double w = (n == 1) ? 1.0 : 0.5;
      y = make_double2(w * a[n - 1].x + 0.5 * a[n + 1].x, w * a[n - 1].y + 0.5 * a[n + 1].y);
    }
    double2 v = g[c * cs + mo + n];
    v.x -= kx * y.y;  // + i kx (y a)
    v.y += kx * y.x;
    if (c == 0) {
      v.x += x[cs + mo + n].x;  // + v
      v.y += x[cs + mo + n].y;
    }
    gl[t] = v;
  }
  __syncthreads();
  const double2* Sm = S + (size_t)mode * C * R;
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    double ar = 0.0, ai = 0.0;
#pragma unroll 8
    for (int col = 0; col < C; ++col) {
      const double2 s = Sm[(size_t)col * R + r];
      const double2 b = gl[col];
      ar += s.x * b.x - s.y * b.y;
      ai += s.x * b.y + s.y * b.x;
    }
    const int c = r / ny;
    const int n = r - c * ny;
    out[c * cs + mo + n] = make_double2(ar, ai);
  }
}

}  // namespace

size_t adv_bytes(const sp_plan* p) {
  const Dims& d = p->d;
  return (size_t)d.nx * d.nzh * 3 * (d.N - 1) * 3 * d.ny * sizeof(double2);
}

sp_status build_advection(sp_plan* p) {
  const Dims& d = p->d;
  const int N = d.N, C = 3 * (N - 1), R = 3 * d.ny;
  const int nmodes = d.nx * d.nzh;
  std::vector<cplx> S((size_t)nmodes * C * R, cplx(0.0, 0.0));
  std::vector<int> work;
  for (int m = 0; m < nmodes; ++m) {
    const int i = m / d.nzh, j = m - i * d.nzh;
    if ((i == 0 && j == 0) || i == d.nx / 2 || j == d.nzh - 1) continue;
    work.push_back(m);
  }
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt == 0 ? 1u : nt, 16u));
  std::vector<int> ok(nt, 1);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (size_t w = t; w < work.size(); w += nt) {
        const int m = work[w];
        const int i = m / d.nzh, j = m - i * d.nzh;
        const int mxv = (i < d.nx / 2) ? i : i - d.nx;
        if (!adv_mode_operator(N, d.alpha * mxv, d.gamma * j, d.re, d.inv_dt,
                               &S[(size_t)m * C * R]))
          ok[t] = 0;
      }
    });
  for (auto& x : th) x.join();
  for (int v : ok)
    if (!v) return set_error(p, SP_ERR_INVALID, "singular advected tau system");
  const size_t bytes = adv_bytes(p);
  if (!p->d_adv) {
    if (hipMalloc((void**)&p->d_adv, bytes) != hipSuccess) {
      p->d_adv = nullptr;
      return set_error(p, SP_ERR_NOMEM, "cannot allocate the advected solve operators");
    }
  }
  if (!p->adv_x) {
    if (hipMalloc((void**)&p->adv_x, (size_t)3 * d.nx * d.nzh * d.ny * sizeof(double2)) !=
        hipSuccess) {
      p->adv_x = nullptr;
      return set_error(p, SP_ERR_NOMEM, "cannot allocate the advected scratch");
    }
  }
  return hip_check(p, hipMemcpy(p->d_adv, S.data(), bytes, hipMemcpyHostToDevice),
                   "upload advected operators");
}

hipError_t launch_adv_apply(sp_plan* p, const double2* g, const double2* x, double2* out) {
  const Dims& d = p->d;
  const size_t sh = (size_t)3 * (d.N - 1) * sizeof(double2);
  SP_PROF_BEGIN(p, KID_ADV);
  hipLaunchKernelGGL(k_adv_apply, dim3(d.nx * d.nzh), dim3(256), sh, p->stream, g, x, p->d_adv,
                     out, d.nx, d.ny, d.nzh, d.alpha);
  SP_PROF_END(p, KID_ADV);
  return hipGetLastError();
}

}  // namespace sp

extern "C" sp_status sp_advected_mode_operator(int32_t N, double kx, double kz, double re,
                                               double inv_dt, double* S_out) {
  if (N < 4 || N > 128 || !S_out || !(re > 0) || !(inv_dt >= 0) || !std::isfinite(kx) ||
      !std::isfinite(kz) || (kx == 0.0 && kz == 0.0))
    return SP_ERR_INVALID;
  return sp::adv_mode_operator(N, kx, kz, re, inv_dt, reinterpret_cast<std::complex<double>*>(S_out))
             ? SP_OK
             : SP_ERR_INVALID;
}

// Host-only numerics of the library (no HIP): the hookstep subproblem of the
// trust-region Newton driver and the per-mode solution operators of the
// implicit step with laminar advection. Kept free of device code so that the
// same file also builds with host sanitizers (tests/test_host_sanitizers.py).
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace sp {

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

static double norm2(const double* v, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += v[i] * v[i];
  return std::sqrt(s);
}

// The damped least-squares solution y(mu) = argmin ||R y - g||^2 + mu ||y||^2
// for the k x k upper-triangular R (column-major, leading dimension ld): the
// rows sqrt(mu) e_i are rotated into R with Givens rotations (no normal
// equations, so the conditioning stays that of R), giving S upper triangular
// with S^T S = R^T R + mu I and z = the rotated right-hand side; y = S^{-1} z
// and q = S^{-T} y (for the Newton correction of mu). S row-major k x k.
static void damped_solve(const double* R, int ld, const double* g, int k, double mu,
                  std::vector<double>& S, std::vector<double>& e, double* z, double* y,
                  double* q) {
  for (int i = 0; i < k; ++i) {
    for (int j = 0; j < i; ++j) S[(size_t)i * k + j] = 0.0;
    for (int j = i; j < k; ++j) S[(size_t)i * k + j] = R[(size_t)j * ld + i];
    z[i] = g[i];
  }
  const double sm = std::sqrt(mu);
  for (int i = 0; i < k; ++i) {
    std::fill(e.begin() + i, e.begin() + k, 0.0);
    e[i] = sm;
    double t = 0.0;  // right-hand side of the extra row
    for (int j = i; j < k; ++j) {
      if (e[j] == 0.0) continue;
      double* Sj = &S[(size_t)j * k];
      const double r = std::hypot(Sj[j], e[j]);
      const double c = Sj[j] / r, s = e[j] / r;
      Sj[j] = r;
      for (int l = j + 1; l < k; ++l) {
        const double a = Sj[l], b = e[l];
        Sj[l] = c * a + s * b;
        e[l] = -s * a + c * b;
      }
      const double zj = z[j];
      z[j] = c * zj + s * t;
      t = -s * zj + c * t;
    }
  }
  for (int i = k - 1; i >= 0; --i) {
    double s2 = z[i];
    const double* Si = &S[(size_t)i * k];
    for (int j = i + 1; j < k; ++j) s2 -= Si[j] * y[j];
    y[i] = s2 / Si[i];
  }
  for (int i = 0; i < k; ++i) {
    double s2 = y[i];
    for (int j = 0; j < i; ++j) s2 -= S[(size_t)j * k + i] * q[j];
    q[i] = s2 / S[(size_t)i * k + i];
  }
}

// The hookstep: y minimising ||g[0..k-1] - R y|| over ||y|| <= delta, given the
// unconstrained minimiser yN. mu from Newton's method on 1/||y(mu)|| = 1/delta
// (Hebden; More & Sorensen), which increases monotonically from mu = 0 when
// ||yN|| > delta. Returns mu; y holds the step.
double hook_solve(const double* R, int ld, const double* g, int k, const double* yN,
                  double delta, double* y) {
  const double nN = norm2(yN, k);
  if (nN <= delta) {
    std::copy(yN, yN + k, y);
    return 0.0;
  }
  std::vector<double> S((size_t)k * k), e(k), z(k), q(k);
  // mu = 0: S = R, y = yN, q = R^{-T} yN
  for (int i = 0; i < k; ++i) {
    double s2 = yN[i];
    for (int j = 0; j < i; ++j) s2 -= R[(size_t)i * ld + j] * q[j];
    q[i] = s2 / R[(size_t)i * ld + i];
  }
  double mu = 0.0, ny = nN, nq = norm2(q.data(), k);
  std::copy(yN, yN + k, y);
  double lo = 0.0, hi = HUGE_VAL;
  for (int it = 0; it < 100; ++it) {
    if (std::fabs(ny - delta) <= 1e-13 * delta) break;
    if (ny > delta) lo = mu; else hi = mu;
    double mn = mu + (ny / nq) * (ny / nq) * (ny - delta) / delta;
    if (!(mn > lo && mn < hi)) mn = std::isfinite(hi) ? 0.5 * (lo + hi) : 2.0 * lo + 1e-300;
    if (mn == mu) break;
    mu = mn;
    damped_solve(R, ld, g, k, mu, S, e, z.data(), y, q.data());
    ny = norm2(y, k);
    nq = norm2(q.data(), k);
  }
  return mu;
}

// ||g[0..k-1] - R y||^2 + g[k]^2: the GMRES model's squared residual at y
double model_res2(const double* R, int ld, const double* g, int k, const double* y) {
  double s = g[k] * g[k];
  for (int i = 0; i < k; ++i) {
    double t = g[i];
    for (int j = i; j < k; ++j) t -= R[(size_t)j * ld + i] * y[j];
    s += t * t;
  }
  return s;
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

extern "C" sp_status sp_hook_step(const double* R, int32_t ld, const double* g, int32_t k,
                                  double delta, double* y, double* mu, double* model_res) {
  if (!R || !g || !y || !mu || !model_res || k < 1 || ld < k || !(delta > 0))
    return SP_ERR_INVALID;
  for (int i = 0; i < k; ++i)
    if (!(R[(size_t)i * ld + i] != 0.0) || !std::isfinite(R[(size_t)i * ld + i]))
      return SP_ERR_INVALID;
  std::vector<double> yN(k);
  for (int i = k - 1; i >= 0; --i) {
    double s2 = g[i];
    for (int j = i + 1; j < k; ++j) s2 -= R[(size_t)j * ld + i] * yN[j];
    yN[i] = s2 / R[(size_t)i * ld + i];
  }
  *mu = sp::hook_solve(R, ld, g, k, yN.data(), delta, y);
  *model_res = std::sqrt(sp::model_res2(R, ld, g, k, y));
  return SP_OK;
}


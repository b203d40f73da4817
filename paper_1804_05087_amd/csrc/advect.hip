// The BEFE step with the laminar advection moved into the implicit operator
// (paper Sec. 3.6, the proposed remedy for the Krylov counts at high Re):
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
#include "host_math.h"
#include "sp_internal.h"

namespace sp {

namespace {

// out_k = S~_k (g_k + i k_x Y x_k + (x_v, 0, 0)) on the used coefficients,
// one block per mode; the mean mode and the Nyquist modes are skipped (their
// output comes from the Stokes solve).
__device__ inline double2 ld_op(const double2* S, size_t i) { return S[i]; }
__device__ inline double2 ld_op(const float2* S, size_t i) {
  const float2 f = S[i];
  return make_double2(f.x, f.y);
}

// S~ in FP64, or its FP32 copy for the mixed-precision path (the sums stay FP64).
template <typename TS>
__global__ void __launch_bounds__(256)
    k_adv_apply(const double2* __restrict__ g, const double2* __restrict__ x,
                const TS* __restrict__ S, double2* __restrict__ out, int nx, int ny,
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
  const TS* Sm = S + (size_t)mode * C * R;
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    double ar = 0.0, ai = 0.0;
#pragma unroll 8
    for (int col = 0; col < C; ++col) {
      const double2 s = ld_op(Sm, (size_t)col * R + r);
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

namespace {

// ---- The same operators built on the device, one workgroup per mode ----

__device__ inline double d1_coef(int n, int m) {  // (D)_{nm}: d/dy on coefficients
  return (m > n && ((m + n) & 1)) ? (n == 0 ? 1.0 : 2.0) * m : 0.0;
}
__device__ inline double d2_coef(int n, int m) {  // (D D)_{nm} = m (m^2 - n^2) / c_n
  return (m >= n + 2 && ((m + n) & 1) == 0)
             ? (double)m * ((double)m * m - (double)n * n) / (n == 0 ? 2.0 : 1.0)
             : 0.0;
}

// Entry (r, c) of the tau matrix that adv_mode_matrix assembles.
__device__ double2 adv_entry(int N, double kx, double kz, double re, double diag, int r, int c) {
  const int n1 = N + 1, V = n1, W = 2 * n1, P = 3 * n1, nm = 3 * (N - 1);
  double er = 0.0, ei = 0.0;
  if (r < nm) {  // momentum component comp on T_n
    const int comp = r / (N - 1), n = r - comp * (N - 1), off = comp * n1;
    if (c >= off && c < off + n1) {
      const int m = c - off;
      er = d2_coef(n, m) / re - (m == n ? diag : 0.0);
      double yc = 0.0;  // coefficient of a_m in (y a)_n
      if (n == 0) {
        if (m == 1) yc = 0.5;
      } else {
        if (m == n - 1) yc = (n == 1) ? 1.0 : 0.5;
        if (m == n + 1) yc = 0.5;
      }
      ei = -kx * yc;
    }
    if (comp == 0) {
      if (c == V + n) er -= 1.0;
      if (c == P + n) er = 0.0, ei = -kx;
    } else if (comp == 1) {
      if (c >= P) er = -d1_coef(n, c - P), ei = 0.0;
    } else {
      if (c == P + n) er = 0.0, ei = -kz;
    }
  } else if (r < nm + 6) {  // no-slip rows: u(1) = 0, u(-1) = 0 for u, v, w
    const int q = r - nm, off = (q >> 1) * n1;
    if (c >= off && c < off + n1) er = (q & 1) ? (((c - off) & 1) ? -1.0 : 1.0) : 1.0;
  } else {  // continuity on T_n
    const int n = r - nm - 6;
    if (c == n) ei = kx;
    else if (c >= V && c < V + n1) er = d1_coef(n, c - V);
    else if (c == W + n) ei = kz;
  }
  return make_double2(er, ei);
}

// Double-double accumulator (Knuth's two-sum and the FMA two-product).
struct DD {
  double hi = 0.0, lo = 0.0;
  __device__ void add(double p, double pe) {
    const double s = hi + p;
    const double bb = s - hi;
    lo += ((hi - (s - bb)) + (p - bb)) + pe;
    hi = s;
  }
  __device__ void add_prod(double a, double b) {
    const double p = a * b;
    add(p, fma(a, b, -p));
  }
};

// X_c <- (LU)^{-1} P X_c (X n x C, row-major) with the workgroup's factors
// and pivots; one thread per column, no barriers. The inner products run over
// every entry (zeros included) so that the unrolled loads overlap instead of
// each waiting on a test of the previous one.
__device__ void adv_lu_solve_col(const double2* __restrict__ LU, const int* piv, int n, int C,
                                 double2* __restrict__ X, int c) {
  for (int k = 0; k < n; ++k) {
    const int p = piv[k];
    if (p != k) {
      const double2 t = X[(size_t)k * C + c];
      X[(size_t)k * C + c] = X[(size_t)p * C + c];
      X[(size_t)p * C + c] = t;
    }
  }
  for (int r = 1; r < n; ++r) {
    double sr = X[(size_t)r * C + c].x, si = X[(size_t)r * C + c].y;
    const double2* Lr = LU + (size_t)r * n;
#pragma unroll 8
    for (int q = 0; q < r; ++q) {
      const double2 l = Lr[q];
      const double2 x = X[(size_t)q * C + c];
      sr -= l.x * x.x - l.y * x.y;
      si -= l.x * x.y + l.y * x.x;
    }
    X[(size_t)r * C + c] = make_double2(sr, si);
  }
  for (int r = n - 1; r >= 0; --r) {
    double sr = X[(size_t)r * C + c].x, si = X[(size_t)r * C + c].y;
    const double2* Ur = LU + (size_t)r * n;
#pragma unroll 8
    for (int q = r + 1; q < n; ++q) {
      const double2 u = Ur[q];
      const double2 x = X[(size_t)q * C + c];
      sr -= u.x * x.x - u.y * x.y;
      si -= u.x * x.y + u.y * x.x;
    }
    const double2 d = Ur[r];
    const double den = d.x * d.x + d.y * d.y;
    X[(size_t)r * C + c] = make_double2((sr * d.x + si * d.y) / den, (si * d.x - sr * d.y) / den);
  }
}

// Row r of -e_c - A x_c accumulated in double-double over the non-zero
// entries of row r only, which the tau matrix's structure fixes: in a
// momentum row n of component comp its own block at m = n - 1, n, n + 1 and
// m = n + 2, n + 4, ... (second derivative), the coupling entries (v and p
// for u, the pressure gradient); all of its block in a no-slip row; u, w and
// the odd-offset derivative of v in a continuity row. The entries come from
// adv_entry, so A is never stored.
__device__ double2 adv_residual_row(int N, double kx, double kz, double re, double diag, int r,
                                    const double2* __restrict__ X, int C, int c) {
  const int n1 = N + 1, V = n1, W = 2 * n1, P = 3 * n1, nm = 3 * (N - 1);
  DD sr, si;
  if (r == c) sr.hi = -1.0;
  auto acc = [&](int q) {
    const double2 a = adv_entry(N, kx, kz, re, diag, r, q);
    const double2 x = X[(size_t)q * C + c];
    sr.add_prod(-a.x, x.x);
    sr.add_prod(a.y, x.y);
    si.add_prod(-a.x, x.y);
    si.add_prod(-a.y, x.x);
  };
  if (r < nm) {
    const int comp = r / (N - 1), n = r - comp * (N - 1), off = comp * n1;
    if (n >= 1) acc(off + n - 1);
    acc(off + n);
    acc(off + n + 1);
    for (int m = n + 2; m <= N; m += 2) acc(off + m);
    if (comp == 0) {
      acc(V + n);
      acc(P + n);
    } else if (comp == 1) {
      for (int m = n + 1; m <= N; m += 2) acc(P + m);
    } else {
      acc(P + n);
    }
  } else if (r < nm + 6) {
    const int off = ((r - nm) >> 1) * n1;
    for (int m = 0; m <= N; ++m) acc(off + m);
  } else {
    const int n = r - nm - 6;
    acc(n);
    for (int m = n + 1; m <= N; m += 2) acc(V + m);
    acc(W + n);
  }
  return make_double2(sr.hi + sr.lo, si.hi + si.lo);
}

// Column c of the operator: solve A x = -e_c with the workgroup's factors,
// refine twice with residuals accumulated in double-double, and write the
// first R rows of x to column c of the mode's operator Sm (R x C, column-major).
__device__ void adv_solve_refine(const double2* __restrict__ LU, const int* piv, int N, double kx,
                                 double kz, double re, double diag, int C, int R,
                                 double2* __restrict__ X, double2* __restrict__ Rw, int c,
                                 double2* __restrict__ Sm) {
  const int n4 = 4 * (N + 1);
  for (int r = 0; r < n4; ++r) X[(size_t)r * C + c] = make_double2(r == c ? -1.0 : 0.0, 0.0);
  adv_lu_solve_col(LU, piv, n4, C, X, c);
  for (int it = 0; it < 2; ++it) {
    for (int r = 0; r < n4; ++r)
      Rw[(size_t)r * C + c] = adv_residual_row(N, kx, kz, re, diag, r, X, C, c);
    adv_lu_solve_col(LU, piv, n4, C, Rw, c);
    for (int r = 0; r < n4; ++r) {
      const double2 x = X[(size_t)r * C + c], d = Rw[(size_t)r * C + c];
      X[(size_t)r * C + c] = make_double2(x.x + d.x, x.y + d.y);
    }
  }
  for (int r = 0; r < R; ++r) Sm[(size_t)c * R + r] = X[(size_t)r * C + c];
}

constexpr int kAdvMaxN4 = 4 * 130;  // ny <= 129

// One workgroup per mode of modes[]: assemble the tau matrix A, LU with
// partial pivoting (the first row of largest modulus, as on the host; only
// the rows with a non-zero multiplier are updated), solve A X = -E for the 3 (N-1) used
// right-hand sides (columns strided over the threads), refine twice with residuals
// accumulated in double-double, and write the first 3 (N+1) rows of X as the
// mode's operator in the layout of k_adv_apply. ws holds, per workgroup,
// LU (n4 x n4) and X and the residual (n4 x C). status[b] = 1 if the
// system is singular.
__global__ void __launch_bounds__(256)
    k_adv_build(const int* __restrict__ modes, int N, int nx, int nzh, double alpha, double gamma,
                double re, double inv_dt, double2* __restrict__ ws, size_t ws_stride,
                double2* __restrict__ S, int* __restrict__ status) {
  __shared__ int piv[kAdvMaxN4];
  __shared__ int rows[kAdvMaxN4];
  __shared__ double bval[256];
  __shared__ int bidx[256];
  __shared__ int nrows;
  const int tid = threadIdx.x;
  const int n1 = N + 1, n4 = 4 * n1, C = 3 * (N - 1), R = 3 * n1;
  const int mode = modes[blockIdx.x];
  const int i = mode / nzh, j = mode - i * nzh;
  const double kx = alpha * ((i < nx / 2) ? i : i - nx), kz = gamma * j;
  const double diag = (kx * kx + kz * kz) / re + inv_dt;
  double2* LU = ws + (size_t)blockIdx.x * ws_stride;
  double2* X = LU + (size_t)n4 * n4;
  double2* Rw = X + (size_t)n4 * C;
  for (int e = tid; e < n4 * n4; e += 256) {
    const int r = e / n4, c = e - r * n4;
    LU[e] = adv_entry(N, kx, kz, re, diag, r, c);
  }
  __syncthreads();
  bool singular = false;
  for (int k = 0; k < n4; ++k) {
    double best = -1.0;
    int bi = n4;
    for (int r = k + tid; r < n4; r += 256) {
      const double2 a = LU[(size_t)r * n4 + k];
      const double v = hypot(a.x, a.y);
      if (v > best) best = v, bi = r;
    }
    bval[tid] = best;
    bidx[tid] = bi;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) {
        const double o = bval[tid + h];
        const int oi = bidx[tid + h];
        if (o > bval[tid] || (o == bval[tid] && oi < bidx[tid])) bval[tid] = o, bidx[tid] = oi;
      }
      __syncthreads();
    }
    const int p = bidx[0];
    const double pv = bval[0];
    __syncthreads();
    if (!(pv > 0.0)) {
      singular = true;
      break;
    }
    if (tid == 0) piv[k] = p, nrows = 0;
    if (p != k)
      for (int c = tid; c < n4; c += 256) {
        const double2 t = LU[(size_t)k * n4 + c];
        LU[(size_t)k * n4 + c] = LU[(size_t)p * n4 + c];
        LU[(size_t)p * n4 + c] = t;
      }
    __syncthreads();
    const double2 akk = LU[(size_t)k * n4 + k];
    const double den = akk.x * akk.x + akk.y * akk.y;
    const double ir = akk.x / den, ii = -akk.y / den;
    // multipliers; the rows with a non-zero one are listed through an LDS
    // counter (their order does not change any result)
    for (int r = k + 1 + tid; r < n4; r += 256) {
      const double2 l = LU[(size_t)r * n4 + k];
      if (l.x != 0.0 || l.y != 0.0) {
        LU[(size_t)r * n4 + k] = make_double2(l.x * ir - l.y * ii, l.x * ii + l.y * ir);
        rows[atomicAdd(&nrows, 1)] = r;
      }
    }
    __syncthreads();
    const int w = n4 - k - 1;
    const int tot = nrows * w;
    for (int e = tid; e < tot; e += 256) {
      const int q = e / w;
      const int c = k + 1 + (e - q * w);
      const int r = rows[q];
      const double2 l = LU[(size_t)r * n4 + k];
      const double2 u = LU[(size_t)k * n4 + c];
      double2 a = LU[(size_t)r * n4 + c];
      a.x -= l.x * u.x - l.y * u.y;
      a.y -= l.x * u.y + l.y * u.x;
      LU[(size_t)r * n4 + c] = a;
    }
    __syncthreads();
  }
  if (singular) {
    if (tid == 0) status[blockIdx.x] = 1;
    return;
  }
  if (tid == 0) status[blockIdx.x] = 0;
  for (int c = tid; c < C; c += 256)
    adv_solve_refine(LU, piv, N, kx, kz, re, diag, C, R, X, Rw, c, S + (size_t)mode * C * R);
}

}  // namespace

__global__ void k_narrow(const double2* __restrict__ a, float2* __restrict__ b, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x)
    b[t] = make_float2((float)a[t].x, (float)a[t].y);
}

// The FP32 copy of the operators used by the mixed-precision path.
static sp_status narrow_adv(sp_plan* p) {
  const size_t n = adv_bytes(p) / sizeof(double2);
  hipLaunchKernelGGL(k_narrow, dim3(4096), dim3(256), 0, p->stream, p->d_adv, p->f_adv, n);
  sp_status s = hip_check(p, hipGetLastError(), "narrow operators");
  if (s) return s;
  return hip_check(p, hipStreamSynchronize(p->stream), "sync");
}

// Allocates the operators (FP64 and the FP32 copy) and the scratch field of
// the advected step if needed.
static sp_status ensure_adv_buffers(sp_plan* p) {
  const Dims& d = p->d;
  if (!p->d_adv) {
    if (hipMalloc((void**)&p->d_adv, adv_bytes(p)) != hipSuccess) {
      p->d_adv = nullptr;
      return set_error(p, SP_ERR_NOMEM, "cannot allocate the advected solve operators");
    }
  }
  if (!p->f_adv) {
    if (hipMalloc((void**)&p->f_adv, adv_bytes(p) / 2) != hipSuccess) {
      p->f_adv = nullptr;
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
  return SP_OK;
}

// The operators of the modes in work built on the device (k_adv_build), in
// chunks whose scratch stays below 4 GiB (freed before returning);
// synchronises.
static sp_status build_advection_device(sp_plan* p, const std::vector<int>& work) {
  const Dims& d = p->d;
  const int N = d.N, n4 = 4 * d.ny, C = 3 * (N - 1);
  if (n4 > kAdvMaxN4) return set_error(p, SP_ERR_INVALID, "ny too large for the device build");
  sp_status s = ensure_adv_buffers(p);
  if (s) return s;
  s = hip_check(p, hipMemsetAsync(p->d_adv, 0, adv_bytes(p), p->stream), "clear operators");
  if (s) return s;
  if (work.empty()) return hip_check(p, hipStreamSynchronize(p->stream), "sync");
  const size_t per_mode = (size_t)n4 * n4 + (size_t)2 * n4 * C;  // double2 entries
  const size_t cap = ((size_t)4 << 30) / (per_mode * sizeof(double2));
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(cap, work.size()));
  // scratch for the build only: the chunk's factors and columns, then the mode
  // list and status
  const size_t ws_bytes = (size_t)chunk * per_mode * sizeof(double2);
  void* scratch = nullptr;
  if (hipMalloc(&scratch, ws_bytes + (work.size() + chunk) * sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(p, SP_ERR_NOMEM, "cannot allocate the scratch of the advected build");
  }
  double2* ws = reinterpret_cast<double2*>(scratch);
  int* d_modes = reinterpret_cast<int*>(reinterpret_cast<char*>(scratch) + ws_bytes);
  int* d_status = d_modes + work.size();
  s = hip_check(p, hipMemcpy(d_modes, work.data(), work.size() * sizeof(int), hipMemcpyHostToDevice),
                "upload modes");
  std::vector<int> st(chunk);
  for (size_t off = 0; s == SP_OK && off < work.size(); off += chunk) {
    const int cnt = (int)std::min<size_t>(chunk, work.size() - off);
    hipLaunchKernelGGL(k_adv_build, dim3(cnt), dim3(256), 0, p->stream, d_modes + off, N, d.nx,
                       d.nzh, d.alpha, d.gamma, d.re, d.inv_dt, ws, per_mode, p->d_adv, d_status);
    s = hip_check(p, hipGetLastError(), "advected build");
    if (s) break;
    s = hip_check(p, hipMemcpyAsync(st.data(), d_status, cnt * sizeof(int), hipMemcpyDeviceToHost,
                                    p->stream),
                  "copy status");
    if (s) break;
    s = hip_check(p, hipStreamSynchronize(p->stream), "sync");
    for (int b = 0; s == SP_OK && b < cnt; ++b)
      if (st[b]) s = set_error(p, SP_ERR_INVALID, "singular advected tau system");
  }
  (void)hipStreamSynchronize(p->stream);  // no launch may still use the scratch
  (void)hipFree(scratch);
  if (s) return s;
  return narrow_adv(p);
}

sp_status build_advection(sp_plan* p) {
  const Dims& d = p->d;
  const int N = d.N, C = 3 * (N - 1), R = 3 * d.ny;
  const int nmodes = d.nx * d.nzh;
  std::vector<int> work;
  for (int m = 0; m < nmodes; ++m) {
    const int i = m / d.nzh, j = m - i * d.nzh;
    if ((i == 0 && j == 0) || i == d.nx / 2 || j == d.nzh - 1) continue;
    work.push_back(m);
  }
  if (!p->adv_host) return build_advection_device(p, work);
  using cplx = std::complex<double>;
  std::vector<cplx> S((size_t)nmodes * C * R, cplx(0.0, 0.0));
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
  sp_status s = ensure_adv_buffers(p);
  if (s) return s;
  s = hip_check(p, hipMemcpy(p->d_adv, S.data(), adv_bytes(p), hipMemcpyHostToDevice),
                "upload advected operators");
  if (s) return s;
  return narrow_adv(p);
}

hipError_t launch_adv_apply(sp_plan* p, const double2* g, const double2* x, double2* out,
                            bool fp32) {
  const Dims& d = p->d;
  const size_t sh = (size_t)3 * (d.N - 1) * sizeof(double2);
  SP_PROF_BEGIN(p, KID_ADV);
  if (fp32)
    hipLaunchKernelGGL(k_adv_apply<float2>, dim3(d.nx * d.nzh), dim3(256), sh, p->stream, g, x,
                       p->f_adv, out, d.nx, d.ny, d.nzh, d.alpha);
  else
    hipLaunchKernelGGL(k_adv_apply<double2>, dim3(d.nx * d.nzh), dim3(256), sh, p->stream, g, x,
                       p->d_adv, out, d.nx, d.ny, d.nzh, d.alpha);
  SP_PROF_END(p, KID_ADV);
  return hipGetLastError();
}

}  // namespace sp


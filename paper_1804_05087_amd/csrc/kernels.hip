// Device kernels of the BEFE step for gfx950 (MI355X).
//
// Data flow of one evaluation (paper Sec. 3.2: derivatives in spectral space,
// products on a physical grid, Chebyshev in y, Fourier in x and z):
//
//  canonical u [3][nx][nz/2+1][ny] (Chebyshev coefficients)
//   --synth_y-->  yv [5][ny][nzm][nx]   values at y_j of u, du/dy, v, w, dw/dy
//   --fft_x_inv-> xp [6][ny][px][nzm]   u, v, w, curl u: x physical (3/2 padded)
//   --z_product-> np [3][ny][px][nzm]   z c2r (padded) . u x omega . z r2c
//   --fft_x_fwd-> nv [3][ny][nzm][nx]   x forward FFT, truncated
//   --analysis_rhs-> g canonical        Chebyshev coefficients + u/dt
//   --stokes_solve-> Phi canonical      per-mode tau/influence-matrix solve (FP64)
//
// nzm = nz/2 (the z Nyquist mode is never stored in intermediates), px = 3nx/2,
// pz = 3nz/2. Every kernel is templated on the real type R of the transform
// path (double, or float for the mixed-precision Jacobian actions); the
// implicit solve is FP64 only.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <type_traits>

#include "device_common.h"
#include "solve_core.h"
#include "solve_row.h"
#include "sp_internal.h"

namespace sp {

// ---------------------------------------------------------------------------
// fft_x_inv: zero-pad lines along x to px and inverse FFT.
// plain == 0: the six output fields u, v, w, omega_x, omega_y, omega_z are
// built from the five y-valued fields (u, du/dy, v, w, dw/dy) with i k_x, i k_z;
// plain != 0: output field f is input field f.
// Block: (y, output field f, chunk of kc z-modes).
// ---------------------------------------------------------------------------
template <typename R, int PT>
__global__ void __launch_bounds__(256)
    k_fft_x_inv(const typename V2<R>::T* __restrict__ yv, typename V2<R>::T* __restrict__ xp,
                const typename V2<R>::T* __restrict__ tw, FFTPlan1D pl, int nx, int ny, int nzm,
                int kc, R alpha, R gamma, int plain) {
  using C = typename V2<R>::T;
  extern __shared__ unsigned char smem_raw[];
  const int px = pl.P;
  const int LS = (PT == 0) ? px : line_stride(PT);
  C* A = reinterpret_cast<C*>(smem_raw);
  C* B = A + kc * LS;
  C* twl = B + kc * LS;
  const int y = blockIdx.x;
  const int f = blockIdx.y;
  const int kz0 = blockIdx.z * kc;
  const int nl = min(kc, nzm - kz0);
  for (int t = threadIdx.x; t < px; t += blockDim.x) twl[t] = tw[t];
  for (int t = threadIdx.x; t < nl * LS; t += blockDim.x) A[t] = mk((R)0, (R)0);
  __syncthreads();
  const size_t fs = (size_t)ny * nzm * nx;  // field stride in yv
    staged_copy<4, C>(
      nl * nx,
      [&](int t) {
        const int l = t / nx;
        const int i = t - l * nx;
        C val = mk((R)0, (R)0);
        if (i == nx / 2) return val;
        const int kz = kz0 + l;
        const int mxv = (i < nx / 2) ? i : i - nx;
        const size_t off = ((size_t)y * nzm + kz) * nx + i;
        const R kxv = alpha * (R)mxv;
        const R kzv = gamma * (R)kz;
        if (plain) {
          val = yv[f * fs + off];
        } else if (f == 0) {
          val = yv[0 * fs + off];
        } else if (f == 1) {
          val = yv[2 * fs + off];
        } else if (f == 2) {
          val = yv[3 * fs + off];
        } else if (f == 3) {  // dw/dy - i kz v
          val = csub(yv[4 * fs + off], sidot(cscale(yv[2 * fs + off], kzv), (R)1));
        } else if (f == 4) {  // i kz u - i kx w
          val = sidot(csub(cscale(yv[0 * fs + off], kzv), cscale(yv[3 * fs + off], kxv)), (R)1);
        } else {  // i kx v - du/dy
          val = csub(sidot(cscale(yv[2 * fs + off], kxv), (R)1), yv[1 * fs + off]);
        }
        return val;
      },
      [&](int t, C v) {
        const int l = t / nx;
        const int i = t - l * nx;
        if (i == nx / 2) return;
        const int pos = (i < nx / 2) ? i : i - nx + px;
        A[lidx<PT>(l, pos, px)] = v;
      });
  __syncthreads();
  C* res = fft_lines<R, PT>(A, B, nl, pl, twl, (R)1);
  #pragma unroll 8
  for (int t = threadIdx.x; t < nl * px; t += blockDim.x) {
    const int x = t / nl;
    const int l = t - x * nl;
    xp[(((size_t)f * ny + y) * px + x) * nzm + kz0 + l] = res[lidx<PT>(l, x, px)];
  }
}

// ---------------------------------------------------------------------------
// z_product: per (y, x) z-line. Fields are paired (u,v), (w,ox), (oy,oz) into
// complex lines a + i b of the Hermitian-extended spectra, inverse FFT gives
// the two real lines at once. mode 0: n = u x omega; mode 1: n = du x Omega +
// U x domega with (U, Omega) from `base`; mode 2: store the six physical
// fields into `base`. The product is packed as (nx + i ny, nz), forward FFT,
// unpacked and scaled by 1/(px pz).
// ---------------------------------------------------------------------------
template <typename R, int PT>
__global__ void __launch_bounds__(256)
    k_z_product(const typename V2<R>::T* __restrict__ xp, typename V2<R>::T* __restrict__ np,
                R* __restrict__ base, const typename V2<R>::T* __restrict__ tw, FFTPlan1D pl,
                int ny, int px, int nzm, int xc, int mode, R scale) {
  using C = typename V2<R>::T;
  extern __shared__ unsigned char smem_raw[];
  const int pz = pl.P;
  const int y = blockIdx.x;
  const int x0 = blockIdx.y * xc;
  const int nxl = min(xc, px - x0);
  const int LS = (PT == 0) ? pz : line_stride(PT);
  C* A = reinterpret_cast<C*>(smem_raw);
  C* B = A + xc * 3 * LS;
  C* twl = B + xc * 3 * LS;
  const size_t fs = (size_t)ny * px * nzm;
  for (int t = threadIdx.x; t < pz; t += blockDim.x) twl[t] = tw[t];
    staged_copy<6, C>(
      nxl * 3 * pz,
      [&](int t) {
        const int m = t % pz;
        const int lj = t / pz;  // x_l * 3 + j
        const int j = lj % 3;
        const int xl = lj / 3;
        const size_t off = ((size_t)y * px + (x0 + xl)) * nzm;
        C val = mk((R)0, (R)0);
        if (m < nzm) {
          C a = xp[(2 * j) * fs + off + m];
          C b = xp[(2 * j + 1) * fs + off + m];
          if (m == 0) {
            a.y = 0;
            b.y = 0;
          }
          val = mk(a.x - b.y, a.y + b.x);
        } else if (m > pz - nzm) {
          const int mm = pz - m;
          C a = conjc(xp[(2 * j) * fs + off + mm]);
          C b = conjc(xp[(2 * j + 1) * fs + off + mm]);
          val = mk(a.x - b.y, a.y + b.x);
        }
        return val;
      },
      [&](int t, C v) { A[lidx<PT>(t / pz, t % pz, pz)] = v; });
  __syncthreads();
  C* res = fft_lines<R, PT>(A, B, nxl * 3, pl, twl, (R)1);
  C* oth = (res == A) ? B : A;
  const size_t bs = (size_t)ny * px * pz;  // base field stride
  #pragma unroll 8
  for (int t = threadIdx.x; t < nxl * pz; t += blockDim.x) {
    const int xl = t / pz;
    const int z = t - xl * pz;
    const C p0 = res[lidx<PT>(xl * 3 + 0, z, pz)];
    const C p1 = res[lidx<PT>(xl * 3 + 1, z, pz)];
    const C p2 = res[lidx<PT>(xl * 3 + 2, z, pz)];
    const R u = p0.x, v = p0.y, w = p1.x, ox = p1.y, oy = p2.x, oz = p2.y;
    const size_t bo = ((size_t)y * px + (x0 + xl)) * pz + z;
    R nxv, nyv, nzv;
    if (mode == 0) {
      nxv = v * oz - w * oy;
      nyv = w * ox - u * oz;
      nzv = u * oy - v * ox;
    } else if (mode == 1) {
      const R U = base[0 * bs + bo], V = base[1 * bs + bo], W = base[2 * bs + bo];
      const R OX = base[3 * bs + bo], OY = base[4 * bs + bo], OZ = base[5 * bs + bo];
      nxv = (v * OZ - w * OY) + (V * oz - W * oy);
      nyv = (w * OX - u * OZ) + (W * ox - U * oz);
      nzv = (u * OY - v * OX) + (U * oy - V * ox);
    } else {
      base[0 * bs + bo] = u;
      base[1 * bs + bo] = v;
      base[2 * bs + bo] = w;
      base[3 * bs + bo] = ox;
      base[4 * bs + bo] = oy;
      base[5 * bs + bo] = oz;
      continue;
    }
    oth[lidx<PT>(xl * 2 + 0, z, pz)] = mk(nxv, nyv);
    oth[lidx<PT>(xl * 2 + 1, z, pz)] = mk(nzv, (R)0);
  }
  if (mode == 2) return;  // uniform across the block
  __syncthreads();
  C* fin = fft_lines<R, PT>(oth, res, nxl * 2, pl, twl, (R)-1);
  const size_t ns = (size_t)ny * px * nzm;
  #pragma unroll 8
  for (int t = threadIdx.x; t < nxl * nzm; t += blockDim.x) {
    const int xl = t / nzm;
    const int m = t - xl * nzm;
    const C a = fin[lidx<PT>(xl * 2 + 0, m, pz)];
    const C am = conjc(fin[lidx<PT>(xl * 2 + 0, (pz - m) % pz, pz)]);
    const C cz = fin[lidx<PT>(xl * 2 + 1, m, pz)];
    const C sx = cscale(cadd(a, am), (R)0.5 * scale);
    const C d = csub(a, am);  // 2 i Ny
    const C sy = mk(d.y * (R)0.5 * scale, -d.x * (R)0.5 * scale);
    const size_t off = ((size_t)y * px + (x0 + xl)) * nzm + m;
    np[0 * ns + off] = sx;
    np[1 * ns + off] = sy;
    np[2 * ns + off] = cscale(cz, scale);
  }
}

// ---------------------------------------------------------------------------
// fft_x_fwd: forward FFT along x of the three product fields, truncation to
// the kept m_x (Nyquist zero). Block: (y, component, chunk of kc z-modes).
// ---------------------------------------------------------------------------
template <typename R, int PT>
__global__ void __launch_bounds__(256)
    k_fft_x_fwd(const typename V2<R>::T* __restrict__ np, typename V2<R>::T* __restrict__ nv,
                const typename V2<R>::T* __restrict__ tw, FFTPlan1D pl, int nx, int ny, int nzm,
                int kc) {
  using C = typename V2<R>::T;
  extern __shared__ unsigned char smem_raw[];
  const int px = pl.P;
  const int LS = (PT == 0) ? px : line_stride(PT);
  C* A = reinterpret_cast<C*>(smem_raw);
  C* B = A + kc * LS;
  C* twl = B + kc * LS;
  const int y = blockIdx.x;
  const int c = blockIdx.y;
  const int kz0 = blockIdx.z * kc;
  const int nl = min(kc, nzm - kz0);
  for (int t = threadIdx.x; t < px; t += blockDim.x) twl[t] = tw[t];
    staged_copy<6, C>(
      nl * px,
      [&](int t) {
        const int x = t / nl;
        const int l = t - x * nl;
        return np[(((size_t)c * ny + y) * px + x) * nzm + kz0 + l];
      },
      [&](int t, C v) {
        const int x = t / nl;
        const int l = t - x * nl;
        A[lidx<PT>(l, x, px)] = v;
      });
  __syncthreads();
  C* res = fft_lines<R, PT>(A, B, nl, pl, twl, (R)-1);
  #pragma unroll 8
  for (int t = threadIdx.x; t < nl * nx; t += blockDim.x) {
    const int l = t / nx;
    const int i = t - l * nx;
    C val = mk((R)0, (R)0);
    if (i != nx / 2) {
      const int pos = (i < nx / 2) ? i : i - nx + px;
      val = res[lidx<PT>(l, pos, px)];
    }
    nv[(((size_t)c * ny + y) * nzm + kz0 + l) * nx + i] = val;
  }
}

// ---------------------------------------------------------------------------
// stokes_solve: per-mode implicit solve (FP64), paper Sec. 2 (the constrained
// inverse of I - dt L) in the Chebyshev-tau / influence-matrix form.
// out = S(g): velocity of (1/Re) Lap phi - phi/dt - grad p = -g, div phi = 0,
// walls (wall_upper, wall_lower) for the (0,0) mode when inhomogeneous, else 0.
// One 64-lane wave per mode, four 16-lane rows (solve_row.h):
//   rows 0, 1: the coupled (v, p) chain with v of parity r (p of the other),
//   rows 2, 3: the decoupled u_perp Helmholtz problem on parity r - 2, swept in
//              the same instruction stream as the Poisson sweep of rows 0, 1.
// (0,0) mode: rows 0, 1 solve for u (parity r), rows 2, 3 for w (parity r - 2).
// Rows without work in a step run it on a dummy array.
// ---------------------------------------------------------------------------
// Orders one wave's LDS accesses between two steps of the solve when no other
// wave of the block takes part: a workgroup-scope fence waits for the wave's
// LDS operations and keeps the compiler from moving any across it.
__device__ inline void lds_order() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup"); }

#define SP_ROW_PAR(par, body)                       \
  _Pragma("unroll") for (int e_ = 0; e_ < E; ++e_) { \
    const int n = (par) + 2 * (l * E + e_);          \
    if (n <= N) {                                    \
      body                                           \
    }                                                \
  }

// AN = 0: the right-hand side g is read from a canonical field. AN = 1 (FP64)
// or 2 (FP32 transform path): g = Tinv nv + xa x is formed here from the
// y-valued product fields nv [3][ny][nz/2][nx] of this mode and the canonical
// field x (a6 fused into a7): the columns are folded into their even and odd
// halves in y (Tinv[n][N-j] = (-1)^n Tinv[n][j]), so each lane forms its
// coefficients n from N/2+1 terms; tinv is the folded half transposed,
// th[j][n] = Tinv[n][j], so the lanes' loads are contiguous.
// Two-wave blocks are held to at most 168 VGPRs (3 waves per SIMD), so that
// every mode's block is resident at once at 48x65x48 (2 x 1128 waves).
// RES (with AN != 0): the residual form of a Jacobian action, out = oa S(g) +
// ob x, written in the Hermitian form: the block of an m_z = 0 mode at m_x > 0
// also writes the conjugate at -m_x (whose block has nothing to do), and the
// (0,0) mode is real. x's entries n <= N are kept in LDS for it.
template <int E, int AN, bool RES = false>
__global__ void __launch_bounds__(AN != 0 ? 128 : 64)
    __attribute__((amdgpu_waves_per_eu(AN != 0 ? 3 : 1)))
    k_stokes_solve(const double2* __restrict__ g, double2* __restrict__ out,
                   const double* __restrict__ modedata, const double* __restrict__ hw_g,
                   int stride, int nx, int ny, int nzh, double alpha, double gamma, double re,
                   double inv_dt, double wu, double wl, int inhomogeneous,
                   const void* __restrict__ nv_raw, const void* __restrict__ tinv_raw,
                   const double2* __restrict__ x, double xa, double oa = 1.0, double ob = 0.0) {
  static_assert(!RES || AN != 0, "the residual form reads x through the fused analysis");
  extern __shared__ unsigned char smem_raw[];
  const int N = ny - 1;
  const int n1 = ny;
  double* rec = reinterpret_cast<double*>(smem_raw);
  double* hw = rec + stride;
  cd* Fpar = reinterpret_cast<cd*>(hw + 3 * n1);
  cd* Fv = Fpar + n1;
  cd* A = Fv + n1;
  cd* divF = A + n1;
  cd* P = divF + n1;
  cd* Rv = P + n1;
  cd* V = Rv + n1;
  cd* Rp = V + n1;
  cd* U = Rp + n1;
  cd* Dm = U + n1;  // output of the idle rows
  const int jh = (ny - 1) / 2 + 1;  // folded column length (AN != 0)
  const int jh8 = (jh + 7) & ~7;    // padded with zeros to whole groups of 8
  // The folded columns of the analysis share the space of the ten arrays
  // above: both waves read them only before the analysis' last barrier, and
  // the arrays are first written after it.
  cd* colE = Fpar;  // [3][jh8] even halves f_j + f_{N-j}
  // odd halves f_j - f_{N-j} ([3][jh8]), 64 bytes past the even ones so that
  // the two addresses an analysis load broadcasts fall in different banks
  cd* colO = colE + 3 * jh8 + 4;
  const int shared_len = (10 * n1 > 6 * jh8 + 4) ? 10 * n1 : 6 * jh8 + 4;
  // [6][64] partial sums of wave 1 (which may still read them after the
  // analysis' last barrier, so they have space of their own)
  double* part_raw = reinterpret_cast<double*>(Fpar + shared_len);
  // x at n <= N for the residual form ([3][n1]), past wave 1's partial sums
  cd* Yx = reinterpret_cast<cd*>(part_raw + 6 * 64);

  // logical order: x mode fastest, so the modes whose product-field entries
  // share a cache line (consecutive m_x at one m_z) run on one XCD
  const int lo = xcd_order(blockIdx.x, gridDim.x);
  const int j = lo / nx;
  const int i = lo - j * nx;
  const int mode = i * nzh + j;
  // With the fused analysis (AN != 0) a mode has two waves: wave 1 loads half of
  // the record and sums half of the analysis' terms, hands its partial sums to
  // wave 0 and leaves; wave 0 does everything else.
  constexpr int NW = (AN != 0) ? 2 : 1;
  const int tid = threadIdx.x & 63;
  const bool shadow = (threadIdx.x >> 6) != 0;
  const int row = tid >> 4;
  const int l = tid & 15;
  const size_t cs = (size_t)nx * nzh * ny;  // component stride
  const size_t mo = ((size_t)i * nzh + j) * ny;
  if constexpr (RES) {
    if (j == 0 && i > nx / 2) return;  // written by its mirror's block (uniform per block)
  }
  const bool nyq = (i == nx / 2) || (j == nzh - 1);
  if (nyq) {
    if (shadow) return;  // uniform per block: both waves leave
    for (int n = tid; n < n1; n += 64) {
      out[mo + n] = make_double2(0.0, 0.0);
      out[cs + mo + n] = make_double2(0.0, 0.0);
      out[2 * cs + mo + n] = make_double2(0.0, 0.0);
    }
    return;
  }
  const int mxv = (i < nx / 2) ? i : i - nx;
  const double kx = alpha * mxv;
  const double kz = gamma * j;
  const double k2 = kx * kx + kz * kz;
  const bool mean = (i == 0 && j == 0);
  const double k = sqrt(k2);
  const double ik = mean ? 0.0 : 1.0 / k;
  const double lam = k2 + re * inv_dt;
  // right-hand side columns first (registers), then the mode record, so the
  // global loads overlap
  double2 ga[3], gb[3], gc[3];
  if constexpr (AN == 0) {
#pragma unroll
    for (int t = 0; t < 3; ++t) {  // clamped loads, masked after (no per-load branches)
      const int n = tid + 64 * t;
      const int nc = n <= N - 2 ? n : N - 2;
      const double keep = n <= N - 2 ? 1.0 : 0.0;
      ga[t] = g[mo + nc];
      gb[t] = g[cs + mo + nc];
      gc[t] = g[2 * cs + mo + nc];
      ga[t] = make_double2(ga[t].x * keep, ga[t].y * keep);
      gb[t] = make_double2(gb[t].x * keep, gb[t].y * keep);
      gc[t] = make_double2(gc[t].x * keep, gc[t].y * keep);
    }
  } else {
    // u/dt part of the right-hand side: issued first, consumed after the analysis
    // (the residual form keeps x up to n = N)
    constexpr int kTop = RES ? 0 : 2;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int n = tid + 64 * t;
      const int nc = n <= N - kTop ? n : N - kTop;
      ga[t] = x[mo + nc];
      gb[t] = x[cs + mo + nc];
      gc[t] = x[2 * cs + mo + nc];
    }
  }
  // fold loads of the y-valued columns (AN != 0) into registers: lane jj takes
  // f_jj and f_{N-jj}; issued before the record loads so both overlap
  using RA = typename std::conditional<AN == 2, float, double>::type;
  using CA = typename V2<RA>::T;
  // folded column entries per lane: jj = tid + 64 q, q < QF; jh <= 64 up to
  // ny = 128 (E <= 4), so only E = 5 needs a second set
  constexpr int QF = (E >= 5) ? 2 : 1;
  CA fa[QF][3], fb[QF][3];
  if constexpr (AN != 0) {
    const CA* nv = reinterpret_cast<const CA*>(nv_raw);
    const int nzm = nzh - 1;
    const size_t cstride = (size_t)ny * nzm * nx;
    const size_t base = (size_t)j * nx + i;
#pragma unroll
    for (int q = 0; q < QF; ++q) {
      const int jj = tid + 64 * q;
      const int jc = jj < jh ? jj : jh - 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        fa[q][c] = nv[c * cstride + (size_t)jc * nzm * nx + base];
        fb[q][c] = nv[c * cstride + (size_t)(N - jc) * nzm * nx + base];
      }
    }
  }
  // mode record and weights (contiguous in LDS: hw = rec + stride) in one round
  // trip: all loads are issued before the first LDS store
  {
    constexpr int RPL = (solve_record_loads(E) + NW - 1) / NW;
    const double* src = modedata + (size_t)mode * stride;
    const int tot = stride + 3 * n1;
    double rv[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int t = threadIdx.x + 64 * NW * q;
      const int tc = t < tot ? t : tot - 1;
      rv[q] = (tc < stride) ? src[tc] : hw_g[tc - stride];
    }
    if constexpr (AN != 0) {
      // even / odd halves, zero padded to jh8 entries
#pragma unroll
      for (int q = 0; q < QF; ++q) {
        const int jj = tid + 64 * q;
        if (jj < jh8 && !shadow) {
          const double in = jj < jh ? 1.0 : 0.0;
          const double same = (jj == N - jj) ? 0.0 : 1.0;  // middle point counted once
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double ar = fa[q][c].x, ai = fa[q][c].y, br = fb[q][c].x, bi = fb[q][c].y;
            colE[c * jh8 + jj] = cd((ar + same * br) * in, (ai + same * bi) * in);
            colO[c * jh8 + jj] = cd((ar - br) * same * in, (ai - bi) * same * in);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int t = threadIdx.x + 64 * NW * q;
      if (t < tot) rec[t] = rv[q];
    }
  }
  if constexpr (AN != 0) {
    // g_n = sum_j Tinv[n][j] f_j + xa x_n for n <= N-2 (the tau rows), one n per lane
    using R = typename std::conditional<AN == 2, float, double>::type;
    const R* Ti = reinterpret_cast<const R*>(tinv_raw);
    __syncthreads();
    const int tmax = (N - 2) / 64 + 1;  // passes over n <= N-2 (uniform)
    // groups of 8 folded terms: wave 0 sums [0, gsplit), wave 1 [gsplit, ng), the
    // larger share to wave 1 (wave 0 also stores the folded columns before, and
    // goes on with the solve after)
    const int ng = jh8 / 8;
    const int gsplit = (NW == 2) ? ng / 2 : ng;
    const int gbeg = shadow ? gsplit : 0;
    const int gend = shadow ? ng : gsplit;
    R* part = reinterpret_cast<R*>(part_raw);  // [6][64] partial sums of wave 1
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if constexpr (RES) {
        const int n = tid + 64 * t;
        if (!shadow && n <= N) {
          Yx[n] = cd(ga[t].x, ga[t].y);
          Yx[n1 + n] = cd(gb[t].x, gb[t].y);
          Yx[2 * n1 + n] = cd(gc[t].x, gc[t].y);
        }
      }
      if (t >= tmax) {
        ga[t] = gb[t] = gc[t] = make_double2(0.0, 0.0);
        continue;
      }
      const int n = tid + 64 * t;
      const int nc = n <= N - 2 ? n : N - 2;
      const cd* src = (nc & 1) ? colO : colE;
      const R* col = Ti + nc;  // th[j][n]: consecutive n across lanes
      R a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0;
      {
        // the table entries of the next group of 8 are loaded while this group
        // is summed (indexes clamped into the table, so the last prefetch is a
        // harmless re-read)
        R tv[8], tn[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          tv[q] = col[(size_t)(8 * gbeg + q < jh ? 8 * gbeg + q : jh - 1) * ny];
        for (int j0 = 8 * gbeg; j0 < 8 * gend; j0 += 8) {  // padded entries are zero
#pragma unroll
          for (int q = 0; q < 8; ++q)
            tn[q] = col[(size_t)(j0 + 8 + q < jh ? j0 + 8 + q : jh - 1) * ny];
#pragma unroll
          for (int h = 0; h < 8; h += 4) {  // two halves of 4 terms (register pressure)
            cd e0[4], e1[4], e2[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              e0[q] = src[j0 + h + q];
              e1[q] = src[jh8 + j0 + h + q];
              e2[q] = src[2 * jh8 + j0 + h + q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              a0r += tv[h + q] * (R)e0[q].re;
              a0i += tv[h + q] * (R)e0[q].im;
              a1r += tv[h + q] * (R)e1[q].re;
              a1i += tv[h + q] * (R)e1[q].im;
              a2r += tv[h + q] * (R)e2[q].re;
              a2i += tv[h + q] * (R)e2[q].im;
            }
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) tv[q] = tn[q];
        }
      }
      if constexpr (NW == 2) {
        if (shadow) {
          part[tid] = a0r;
          part[64 + tid] = a0i;
          part[128 + tid] = a1r;
          part[192 + tid] = a1i;
          part[256 + tid] = a2r;
          part[320 + tid] = a2i;
        }
        __syncthreads();
        a0r += part[tid];
        a0i += part[64 + tid];
        a1r += part[128 + tid];
        a1i += part[192 + tid];
        a2r += part[256 + tid];
        a2i += part[320 + tid];
        if (t + 1 < tmax) __syncthreads();  // the next pass rewrites part (uniform)
      }
      const double keep = n <= N - 2 ? 1.0 : 0.0;
      const double2 x0 = ga[t], x1 = gb[t], x2 = gc[t];
      ga[t] = make_double2(((double)a0r + xa * x0.x) * keep, ((double)a0i + xa * x0.y) * keep);
      gb[t] = make_double2(((double)a1r + xa * x1.x) * keep, ((double)a1i + xa * x1.y) * keep);
      gc[t] = make_double2(((double)a2r + xa * x2.x) * keep, ((double)a2i + xa * x2.y) * keep);
    }
  }
  // wave 1's part ended with the analysis' last barrier (it is uniform per wave):
  // from here on one wave works, and its steps exchange data through LDS,
  // ordered by lds_order() instead of barriers
  if (shadow) return;
  {
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int n = tid + 64 * t;
      if (n < n1) {
        const cd fu(re * ga[t].x, re * ga[t].y);
        const cd fv(re * gb[t].x, re * gb[t].y);
        const cd fw(re * gc[t].x, re * gc[t].y);
        if (mean) {
          Rv[n] = -fu;  // (0,0): u and w solve Dirichlet Helmholtz problems
          Rp[n] = -fw;
        } else {
          Fpar[n] = (fu * kx + fw * kz) * ik;
          Rp[n] = -((fu * kz - fw * kx) * ik);  // -F_perp
          Fv[n] = fv;
        }
      }
    }
  }
  lds_order();
  const ModeLayout L{n1};
  const SweepRec helm(rec + L.helm(), n1, lam);
  const SweepRec pois(rec + L.pois(), n1, k2);
  const bool vrow = row < 2;
  const int pv = row & 1;  // v parity (rows 0, 1), u_perp / w parity (rows 2, 3)
  const int po = 1 - pv;
  if (mean) {
    cd bu(0.0);
    if (inhomogeneous && vrow) bu = cd(pv == 0 ? 0.5 * (wu + wl) : 0.5 * (wu - wl));
    wsweep<E>(helm, hw, N, pv, vrow ? Rv : Rp, bu, vrow ? P : U, l);
  } else {
    // divF = i k F_par + D F_v on rows 0, 1, formed as the derivative is stored
    // (rows 2, 3 differentiate into the idle array: a per-lane select, no branch)
    wderiv<E>(N, pv, vrow ? Fv : Rp, vrow ? divF : Dm, l, [&](int m, cd v) {
      const cd t = mul_i(Fpar[m] * k) + v;
      return vrow ? t : v;
    });
    lds_order();
    // P = Pois(div F) on rows 0, 1; U = Helm(-F_perp) on rows 2, 3
    wsweep<E>(vrow ? pois : helm, hw, N, vrow ? po : pv, vrow ? divF : Rp, cd(0.0), vrow ? P : U,
              l);
    lds_order();
    // Rv = D P - F_v on rows 0, 1, formed as the derivative is stored
    wderiv<E>(N, po, vrow ? P : Rp, vrow ? Rv : Dm, l, [&](int m, cd v) {
      const cd t = v - Fv[m];
      return vrow ? t : v;
    });
    lds_order();
    wsweep<E>(helm, hw, N, pv, vrow ? Rv : Rp, cd(0.0), vrow ? V : Dm, l);
    lds_order();
    // influence correction: (c_delta, c_b) = -Minv (D v(1), tau definition)
    cd ca(0.0), cb(0.0);
    {
      cd la(0.0);
      SP_ROW_PAR(pv, la = la + V[n] * ((double)n * n);)
      la = row_sum(la);
      const int m = (N % 2 == pv) ? N : N - 1;
      cd lb = V[m] * lam;
      if (m == N - 1) lb = lb + P[N] * (2.0 * N);
      const double* Mi = rec + L.minv() + 4 * pv;
      ca = -(la * Mi[0] + lb * Mi[1]);
      cb = -(la * Mi[2] + lb * Mi[3]);
    }
    const double* vdel = rec + L.vdel();
    const double* vb = rec + L.vb();
    lds_order();
    // V += c_delta vdel + c_b vb on rows 0, 1, taken as the derivative loads V (the
    // lane that owns n updates it and stores it back for the output)
    wderiv<E>(N, pv, vrow ? V : Rp, vrow ? A : Dm, l, StoreDeriv(), [&](int n, cd v, bool own) {
      const cd t = v + ca * vdel[n] + cb * vb[n];
      if (vrow && own) V[n] = t;
      return vrow ? t : v;
    });
  }
  lds_order();
  // n1 <= 32 E coefficients: a fixed, unrolled pass count, so the LDS reads of
  // every pass are issued together
#pragma unroll
  for (int q = 0; q < (32 * E + 63) / 64; ++q) {
    const int n = tid + 64 * q;
    if (n >= n1) break;
    cd uo, vo, wo;
    if (mean) {
      uo = P[n];
      wo = U[n];
    } else {
      const cd upar = mul_i(A[n]) * ik;
      uo = (upar * kx + U[n] * kz) * ik;
      wo = (upar * kz - U[n] * kx) * ik;
      vo = V[n];
    }
    if constexpr (RES) {
      uo = uo * oa + Yx[n] * ob;
      vo = vo * oa + Yx[n1 + n] * ob;
      wo = wo * oa + Yx[2 * n1 + n] * ob;
      if (mean) uo.im = vo.im = wo.im = 0.0;
    }
    out[mo + n] = make_double2(uo.re, uo.im);
    out[cs + mo + n] = make_double2(vo.re, vo.im);
    out[2 * cs + mo + n] = make_double2(wo.re, wo.im);
    if constexpr (RES) {
      if (j == 0 && i > 0) {  // 0 < m_x < nx/2: its mirror at -m_x
        const size_t mm = (size_t)(nx - i) * nzh * ny;
        out[mm + n] = make_double2(uo.re, -uo.im);
        out[cs + mm + n] = make_double2(vo.re, -vo.im);
        out[2 * cs + mm + n] = make_double2(wo.re, -wo.im);
      }
    }
  }
}

// out = a x + b y (x or y may be NULL, meaning zero)
__global__ void k_axpby(const double2* __restrict__ x, double a, const double2* __restrict__ y,
                        double b, double2* __restrict__ out, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    double rx = 0, ix = 0;
    if (x) {
      rx = a * x[t].x;
      ix = a * x[t].y;
    }
    if (y) {
      rx += b * y[t].x;
      ix += b * y[t].y;
    }
    out[t] = make_double2(rx, ix);
  }
}

// Per-block partial sums of (1/2) sum_modes w_m sum_c a^H G a (volume-normalised
// squared L2 norm), w_m = 1 (m_z = 0) or 2 (m_z > 0), Nyquist excluded, with the
// Chebyshev Gram matrix G_nm = int T_n T_m dy (zero for n + m odd; the plan's
// table, row-major). One wave per column (component, mode): lane n forms
// (G a)_n from the column's entries of its parity, then a_n^* (G a)_n is
// reduced over the wave; four columns per block at a time.
__global__ void __launch_bounds__(256)
    k_norm_partial(const double2* __restrict__ a, const double* __restrict__ G,
                   double* __restrict__ partial, int nx, int ny, int nzh) {
  __shared__ double red[4];
  const int ncol = 3 * nx * nzh;
  const int wid = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  for (int col = blockIdx.x * 4 + wid; col < ncol; col += gridDim.x * 4) {  // wave-uniform
    const int j = col % nzh;
    const int i = (col / nzh) % nx;
    if (i == nx / 2 || j == nzh - 1) continue;
    const double2* v = a + (size_t)col * ny;
    double s = 0.0;
    for (int n = lane; n < ny; n += 64) {
      const double* g = G + (size_t)n * ny;
      double tr = 0.0, ti = 0.0;
      for (int m = (n & 1); m < ny; m += 2) {
        const double2 vm = v[m];
        tr += g[m] * vm.x;
        ti += g[m] * vm.y;
      }
      const double2 vn = v[n];
      s += vn.x * tr + vn.y * ti;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    acc += (j == 0 ? 1.0 : 2.0) * s;
  }
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = 0.5 * (red[0] + red[1] + red[2] + red[3]);
}

// Packed real vector <-> canonical (see sp.h for the order).
__global__ void k_pack(const double2* __restrict__ c, double* __restrict__ packed, int nx, int ny,
                       int nzh) {
  const int nz = 2 * (nzh - 1);
  const int per_n = (nx - 1) * (nz - 1);  // reals per (component, n)
  const int total = 3 * ny * per_n;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const int cn = t / per_n;
    const int r = t - cn * per_n;
    const int comp = cn / ny;
    const int n = cn - comp * ny;
    int i, j, part;
    if (r == 0) {
      i = 0; j = 0; part = 0;
    } else if (r < 1 + 2 * (nx / 2 - 1)) {
      const int q = r - 1;
      i = 1 + q / 2; j = 0; part = q & 1;
    } else {
      const int q = r - 1 - 2 * (nx / 2 - 1);
      const int mi = q / 2;  // index over (j - 1, i without Nyquist)
      part = q & 1;
      j = 1 + mi / (nx - 1);
      int ii = mi % (nx - 1);
      i = (ii < nx / 2) ? ii : ii + 1;
    }
    const double2 v = c[(((size_t)comp * nx + i) * nzh + j) * ny + n];
    packed[t] = part ? v.y : v.x;
  }
}

__global__ void k_unpack(const double* __restrict__ packed, double2* __restrict__ c, int nx,
                         int ny, int nzh) {
  const int nz = 2 * (nzh - 1);
  const size_t total = (size_t)3 * nx * nzh * ny;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const int n = t % ny;
    const int j = (t / ny) % nzh;
    const int i = (t / ((size_t)ny * nzh)) % nx;
    const int comp = t / ((size_t)ny * nzh * nx);
    const size_t cbase = ((size_t)comp * ny + n) * (size_t)((nx - 1) * (nz - 1));
    double2 v = make_double2(0.0, 0.0);
    if (i != nx / 2 && j != nzh - 1) {
      if (j == 0) {
        if (i == 0) {
          v = make_double2(packed[cbase], 0.0);
        } else {
          const int ip = (i < nx / 2) ? i : nx - i;
          const size_t o = cbase + 1 + 2 * (ip - 1);
          v = make_double2(packed[o], packed[o + 1]);
          if (i > nx / 2) v.y = -v.y;
        }
      } else {
        const int ii = (i < nx / 2) ? i : i - 1;
        const size_t o = cbase + 1 + 2 * (nx / 2 - 1) + 2 * ((size_t)(j - 1) * (nx - 1) + ii);
        v = make_double2(packed[o], packed[o + 1]);
      }
    }
    c[t] = v;
  }
}

// ----------------------------------- launchers -----------------------------------

// Calls LAUNCH(P) with P a supported compile-time FFT length, or 0.
#define SP_FFT_DISPATCH(PV, LAUNCH) \
  switch (PV) {                     \
    case 12: LAUNCH(12); break;     \
    case 24: LAUNCH(24); break;     \
    case 36: LAUNCH(36); break;     \
    case 48: LAUNCH(48); break;     \
    case 72: LAUNCH(72); break;     \
    case 96: LAUNCH(96); break;     \
    case 144: LAUNCH(144); break;   \
    case 192: LAUNCH(192); break;   \
    default: LAUNCH(0); break;      \
  }

// LDS elements per FFT line (padded layout for the specialised lengths).
static int lds_line(int P) { return fft_length_specialised(P) ? line_stride(P) : P; }

static int chunk_for(int P, int total, size_t elem) {
  // largest chunk whose two ping-pong buffers (plus twiddles) fit in 48 KiB of LDS
  const int L = lds_line(P);
  int k = (int)((48 * 1024 - P * elem) / (2 * L * elem));
  if (k < 1) k = 1;
  if (k > total) k = total;
  return k;
}

// LDS Stockham fallbacks for x lengths without a register kernel (xline.hip)
hipError_t launch_fft_x_inv_lds(sp_plan* p, const void* in, void* out, int nfields, int plain,
                                bool fp32) {
  const Dims& d = p->d;
  const size_t el = fp32 ? sizeof(float2) : sizeof(double2);
  const int kc = chunk_for(d.px, d.nzm, el);
  dim3 grid(d.ny, nfields, (d.nzm + kc - 1) / kc);
  const size_t sh = (2 * (size_t)kc * lds_line(d.px) + d.px) * el;
  SP_PROF_BEGIN(p, KID_FFT_X_INV);
#define L32(PV)                                                                                 \
  hipLaunchKernelGGL((k_fft_x_inv<float, PV>), grid, dim3(256), sh, p->stream, (const float2*)in, \
                     (float2*)out, p->f_twx, p->fx, d.nx, d.ny, d.nzm, kc, (float)d.alpha,      \
                     (float)d.gamma, plain)
#define L64(PV)                                                                          \
  hipLaunchKernelGGL((k_fft_x_inv<double, PV>), grid, dim3(256), sh, p->stream,          \
                     (const double2*)in, (double2*)out, p->d_twx, p->fx, d.nx, d.ny, d.nzm, kc, \
                     d.alpha, d.gamma, plain)
  if (fp32) {
    SP_FFT_DISPATCH(d.px, L32)
  } else {
    SP_FFT_DISPATCH(d.px, L64)
  }
#undef L32
#undef L64
  SP_PROF_END(p, KID_FFT_X_INV);
  return hipGetLastError();
}

// LDS Stockham fallback for z lengths without a register kernel (zline.hip)
hipError_t launch_z_product_lds(sp_plan* p, int mode, bool fp32) {
  const Dims& d = p->d;
  const size_t el = fp32 ? sizeof(float2) : sizeof(double2);
  int xc = (int)((48 * 1024 - d.pz * el) / (2 * 3 * lds_line(d.pz) * el));
  if (xc < 1) xc = 1;
  if (xc > d.px) xc = d.px;
  dim3 grid(d.ny, (d.px + xc - 1) / xc);
  const size_t sh = (2 * (size_t)xc * 3 * lds_line(d.pz) + d.pz) * el;
  const double scale = 1.0 / ((double)d.px * d.pz);
  SP_PROF_BEGIN(p, KID_Z_PRODUCT);
#define L32(PV)                                                                                  \
  hipLaunchKernelGGL((k_z_product<float, PV>), grid, dim3(256), sh, p->stream,                   \
                     (const float2*)p->xp, (float2*)p->np, p->base32, p->f_twz, p->fz, d.ny, d.px, \
                     d.nzm, xc, mode, (float)scale)
#define L64(PV)                                                                                   \
  hipLaunchKernelGGL((k_z_product<double, PV>), grid, dim3(256), sh, p->stream,                   \
                     (const double2*)p->xp, (double2*)p->np, p->base, p->d_twz, p->fz, d.ny, d.px, \
                     d.nzm, xc, mode, scale)
  if (fp32) {
    SP_FFT_DISPATCH(d.pz, L32)
  } else {
    SP_FFT_DISPATCH(d.pz, L64)
  }
#undef L32
#undef L64
  SP_PROF_END(p, KID_Z_PRODUCT);
  return hipGetLastError();
}

hipError_t launch_fft_x_fwd_lds(sp_plan* p, const void* in, void* out, int nfields, bool fp32) {
  const Dims& d = p->d;
  const size_t el = fp32 ? sizeof(float2) : sizeof(double2);
  const int kc = chunk_for(d.px, d.nzm, el);
  dim3 grid(d.ny, nfields, (d.nzm + kc - 1) / kc);
  const size_t sh = (2 * (size_t)kc * lds_line(d.px) + d.px) * el;
  SP_PROF_BEGIN(p, KID_FFT_X_FWD);
#define L32(PV)                                                                                 \
  hipLaunchKernelGGL((k_fft_x_fwd<float, PV>), grid, dim3(256), sh, p->stream, (const float2*)in, \
                     (float2*)out, p->f_twx, p->fx, d.nx, d.ny, d.nzm, kc)
#define L64(PV)                                                                       \
  hipLaunchKernelGGL((k_fft_x_fwd<double, PV>), grid, dim3(256), sh, p->stream,       \
                     (const double2*)in, (double2*)out, p->d_twx, p->fx, d.nx, d.ny, d.nzm, kc)
  if (fp32) {
    SP_FFT_DISPATCH(d.px, L32)
  } else {
    SP_FFT_DISPATCH(d.px, L64)
  }
#undef L32
#undef L64
  SP_PROF_END(p, KID_FFT_X_FWD);
  return hipGetLastError();
}

// elements per lane of a 16-lane row covering one parity chain (ny <= 129)
int solve_lanes_per_chain(int ny) { return ((ny - 1) / 2 + 1 + 15) / 16; }

static size_t solve_lds_bytes(const sp_plan* p, bool fused, bool res = false) {
  const Dims& d = p->d;
  const size_t jh8 = (((d.ny - 1) / 2 + 1) + 7) & ~7;
  // ten arrays of ny entries, which the fused analysis' folded columns share
  const size_t arrays = fused ? std::max<size_t>(10 * (size_t)d.ny, 6 * jh8 + 4) : 10 * (size_t)d.ny;
  return (size_t)p->mode_stride * sizeof(double) + 3 * (size_t)d.ny * sizeof(double) +
         arrays * sizeof(cd) + (fused ? 6 * 64 * sizeof(double) : 0) +
         (res ? 3 * (size_t)d.ny * sizeof(cd) : 0);
}

#define SP_SOLVE_DISPATCH(LAUNCH)                   \
  switch (solve_lanes_per_chain(p->d.ny)) {         \
    case 1: LAUNCH(1); break;                       \
    case 2: LAUNCH(2); break;                       \
    case 3: LAUNCH(3); break;                       \
    case 4: LAUNCH(4); break;                       \
    default: LAUNCH(5); break;                      \
  }

hipError_t launch_stokes_solve(sp_plan* p, const double2* g, double2* out, int inhomogeneous) {
  const Dims& d = p->d;
  const size_t sh = solve_lds_bytes(p, false);
  SP_PROF_BEGIN(p, KID_SOLVE);
#define SP_SOLVE_LAUNCH(EV)                                                                     \
  hipLaunchKernelGGL((k_stokes_solve<EV, 0>), dim3(d.nx * d.nzh), dim3(64), sh, p->stream, g,   \
                     out, p->d_mode, p->d_hw, p->mode_stride, d.nx, d.ny, d.nzh, d.alpha,       \
                     d.gamma, d.re, d.inv_dt, d.wall_upper, d.wall_lower, inhomogeneous, nullptr, \
                     nullptr, nullptr, 0.0)
  SP_SOLVE_DISPATCH(SP_SOLVE_LAUNCH)
#undef SP_SOLVE_LAUNCH
  SP_PROF_END(p, KID_SOLVE);
  return hipGetLastError();
}

// Chebyshev analysis of p->nv fused into the solve: out = S(Tinv nv + xa x).
hipError_t launch_analysis_solve(sp_plan* p, const double2* x, double xa, double2* out,
                                 int inhomogeneous, bool fp32) {
  const Dims& d = p->d;
  const size_t sh = solve_lds_bytes(p, true);
  SP_PROF_BEGIN(p, KID_SOLVE);
#define SP_SOLVE_LAUNCH(EV)                                                                       \
  if (fp32)                                                                                       \
    hipLaunchKernelGGL((k_stokes_solve<EV, 2>), dim3(d.nx * d.nzh), dim3(128), sh, p->stream,      \
                       nullptr, out, p->d_mode, p->d_hw, p->mode_stride, d.nx, d.ny, d.nzh,      \
                       d.alpha, d.gamma, d.re, d.inv_dt, d.wall_upper, d.wall_lower,             \
                       inhomogeneous, p->nv, p->f_tinv_th, x, xa, 1.0, 0.0);                         \
  else                                                                                            \
    hipLaunchKernelGGL((k_stokes_solve<EV, 1>), dim3(d.nx * d.nzh), dim3(128), sh, p->stream,      \
                       nullptr, out, p->d_mode, p->d_hw, p->mode_stride, d.nx, d.ny, d.nzh,      \
                       d.alpha, d.gamma, d.re, d.inv_dt, d.wall_upper, d.wall_lower,             \
                       inhomogeneous, p->nv, p->d_tinv_th, x, xa, 1.0, 0.0)
  SP_SOLVE_DISPATCH(SP_SOLVE_LAUNCH)
#undef SP_SOLVE_LAUNCH
  SP_PROF_END(p, KID_SOLVE);
  return hipGetLastError();
}

// The residual form of the same: out = oa S(Tinv nv + xa x) + ob x in the
// Hermitian form, homogeneous walls.
hipError_t launch_analysis_solve_res(sp_plan* p, const double2* x, double xa, double oa, double ob,
                                     double2* out, bool fp32) {
  const Dims& d = p->d;
  const size_t sh = solve_lds_bytes(p, true, true);
  SP_PROF_BEGIN(p, KID_SOLVE);
#define SP_SOLVE_LAUNCH(EV)                                                                       \
  if (fp32)                                                                                       \
    hipLaunchKernelGGL((k_stokes_solve<EV, 2, true>), dim3(d.nx * d.nzh), dim3(128), sh,           \
                       p->stream, nullptr, out, p->d_mode, p->d_hw, p->mode_stride, d.nx, d.ny,  \
                       d.nzh, d.alpha, d.gamma, d.re, d.inv_dt, d.wall_upper, d.wall_lower, 0,   \
                       p->nv, p->f_tinv_th, x, xa, oa, ob);                                      \
  else                                                                                            \
    hipLaunchKernelGGL((k_stokes_solve<EV, 1, true>), dim3(d.nx * d.nzh), dim3(128), sh,           \
                       p->stream, nullptr, out, p->d_mode, p->d_hw, p->mode_stride, d.nx, d.ny,  \
                       d.nzh, d.alpha, d.gamma, d.re, d.inv_dt, d.wall_upper, d.wall_lower, 0,   \
                       p->nv, p->d_tinv_th, x, xa, oa, ob)
  SP_SOLVE_DISPATCH(SP_SOLVE_LAUNCH)
#undef SP_SOLVE_LAUNCH
  SP_PROF_END(p, KID_SOLVE);
  return hipGetLastError();
}

hipError_t launch_axpby(sp_plan* p, const double2* x, double a, const double2* y, double b,
                        double2* out, size_t n) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  SP_PROF_BEGIN(p, KID_AXPBY);
  hipLaunchKernelGGL(k_axpby, dim3(blocks), dim3(256), 0, p->stream, x, a, y, b, out, n);
  SP_PROF_END(p, KID_AXPBY);
  return hipGetLastError();
}

hipError_t launch_norm_partial(sp_plan* p, const double2* a, double* partial, int* nblocks) {
  const Dims& d = p->d;
  const int ncol = 3 * d.nx * d.nzh;
  int blocks = (ncol + 3) / 4;  // one wave per column
  if (blocks > p->npartial) blocks = p->npartial;
  SP_PROF_BEGIN(p, KID_NORM);
  hipLaunchKernelGGL(k_norm_partial, dim3(blocks), dim3(256), 0, p->stream, a, p->d_G, partial,
                     d.nx, d.ny, d.nzh);
  *nblocks = blocks;
  SP_PROF_END(p, KID_NORM);
  return hipGetLastError();
}

hipError_t launch_pack(sp_plan* p, const double2* c, double* packed) {
  const Dims& d = p->d;
  const int total = 3 * d.ny * (d.nx - 1) * (d.nz - 1);
  int blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  SP_PROF_BEGIN(p, KID_PACK);
  hipLaunchKernelGGL(k_pack, dim3(blocks), dim3(256), 0, p->stream, c, packed, d.nx, d.ny, d.nzh);
  SP_PROF_END(p, KID_PACK);
  return hipGetLastError();
}

hipError_t launch_unpack(sp_plan* p, const double* packed, double2* c) {
  const Dims& d = p->d;
  const size_t total = (size_t)3 * d.nx * d.nzh * d.ny;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  SP_PROF_BEGIN(p, KID_UNPACK);
  hipLaunchKernelGGL(k_unpack, dim3(blocks), dim3(256), 0, p->stream, packed, c, d.nx, d.ny,
                     d.nzh);
  SP_PROF_END(p, KID_UNPACK);
  return hipGetLastError();
}

}  // namespace sp

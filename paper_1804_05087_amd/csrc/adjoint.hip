// Vector-Jacobian products: the adjoint of the linearised BEFE step.
//
// With S_0 the homogeneous implicit solve and N_U(du) = du x Omega + U x curl(du),
// J_Phi du = S_0(du/dt + N_U du). Its adjoint in the Parseval inner product
// <a, b> = sum over stored modes of w_m Re(conj(a) . b) (w_m = 1 for m_z = 0,
// 2 for m_z > 0) is
//   J_Phi^+ w = a/dt + N_U^+ a,  a = S_0^+ w,
// where every stage is replaced by its adjoint in reverse order:
//   S_0^+        : per mode, the transposed influence-matrix/tau solve (FP64)
//   analysis^+   : Tinv^T along y
//   truncate+FFT^+ : zero-pad + inverse FFT (scaled by 1/(px pz))
//   product^+    : du_bar = Omega x lam, dw_bar = lam x U (physical space)
//   pad+iFFT^+   : forward FFT + truncation
//   curl/synth^+ : conj(i k) factors and T^T, (T.D)^T along y.
// The packed-Euclidean adjoint used by GMRES and autograd follows by scaling
// the (0,0) mode (counted once in the packed vector, its Parseval weight is 1
// while every other stored mode carries half of a conjugate pair).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "solve_core.h"
#include "solve_row.h"
#include "sp_internal.h"

namespace sp {

// ---------------------------------------------------------------------------
// stokes_solve_adj: out = S_0^+ w per mode (conjugate transpose of the solve
// with homogeneous walls): the forward steps of k_stokes_solve transposed and
// taken in reverse order. One 64-lane wave per mode, four 16-lane rows:
// rows 0, 1 run the (v, p) chain with v of parity r, rows 2, 3 the u_perp
// chain of parity r - 2, whose transposed Helmholtz sweep shares a step with
// the v sweep of rows 0, 1. (0,0) mode: rows 0, 1 u, rows 2, 3 w.
// ---------------------------------------------------------------------------
#define SP_ROW_PAR(par, body)                       \
  _Pragma("unroll") for (int e_ = 0; e_ < E; ++e_) { \
    const int n = (par) + 2 * (l * E + e_);          \
    if (n <= N) {                                    \
      body                                           \
    }                                                \
  }

template <int E>
__global__ void __launch_bounds__(64)
    k_stokes_solve_adj(const double2* __restrict__ w, double2* __restrict__ out,
                       const double* __restrict__ modedata, const double* __restrict__ hw_g,
                       int stride, int nx, int ny, int nzh, double alpha, double gamma, double re,
                       double inv_dt) {
  extern __shared__ unsigned char smem_raw[];
  const int N = ny - 1;
  const int n1 = ny;
  double* rec = reinterpret_cast<double*>(smem_raw);
  double* hw = rec + stride;
  cd* Upb = reinterpret_cast<cd*>(hw + 3 * n1);  // adjoint of u_par
  cd* Ub = Upb + n1;                              // adjoint of u_perp
  cd* Vb = Ub + n1;                               // adjoint of v
  cd* A = Vb + n1;
  cd* Tm = A + n1;
  cd* W = Tm + n1;    // scratch of rows 0, 1
  cd* W2 = W + n1;    // scratch of rows 2, 3
  cd* Rb = W2 + n1;
  cd* Rb2 = Rb + n1;
  cd* Pb = Rb2 + n1;
  cd* Db = Pb + n1;
  cd* Fpb = Db + n1;
  cd* Fpp = Fpb + n1;
  cd* Fvb = Fpp + n1;
  cd* Dm = Fvb + n1;  // output of the idle rows

  const int mode = blockIdx.x;
  const int i = mode / nzh;
  const int j = mode - i * nzh;
  const int tid = threadIdx.x;
  const int row = tid >> 4;
  const int l = tid & 15;
  const size_t cs = (size_t)nx * nzh * ny;
  const size_t mo = ((size_t)i * nzh + j) * ny;
  const bool nyq = (i == nx / 2) || (j == nzh - 1);
  if (nyq) {
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
  double2 wa[3], wb[3], wc[3];
  // packed-Euclidean -> Parseval weights: the (0,0) mode counts twice
  const double wscale = mean ? 2.0 : 1.0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {  // clamped loads, masked after (no per-load branches)
    const int n = tid + 64 * t;
    const int nc = n < n1 ? n : N;
    const double keep = n < n1 ? wscale : 0.0;
    wa[t] = w[mo + nc];
    wb[t] = w[cs + mo + nc];
    wc[t] = w[2 * cs + mo + nc];
    wa[t] = make_double2(wa[t].x * keep, wa[t].y * keep);
    wb[t] = make_double2(wb[t].x * keep, wb[t].y * keep);
    wc[t] = make_double2(wc[t].x * keep, wc[t].y * keep);
  }
  // mode record and weights (contiguous in LDS: hw = rec + stride) in one round
  // trip: all loads are issued before the first LDS store
  {
    constexpr int RPL = solve_record_loads(E);
    const double* src = modedata + (size_t)mode * stride;
    const int tot = stride + 3 * n1;
    double rv[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int t = tid + 64 * q;
      const int tc = t < tot ? t : tot - 1;
      rv[q] = (tc < stride) ? src[tc] : hw_g[tc - stride];
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int t = tid + 64 * q;
      if (t < tot) rec[t] = rv[q];
    }
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int n = tid + 64 * t;
    if (n < n1) {
      const cd ub(wa[t].x, wa[t].y), vb(wb[t].x, wb[t].y), wbv(wc[t].x, wc[t].y);
      if (mean) {
        Upb[n] = ub;
        Ub[n] = wbv;
      } else {
        Upb[n] = (ub * kx + wbv * kz) * ik;
        Ub[n] = (ub * kz - wbv * kx) * ik;
      }
      Vb[n] = vb;
      Pb[n] = cd(0.0);
      Fvb[n] = cd(0.0);
      Fpb[n] = cd(0.0);
      Fpp[n] = cd(0.0);
    }
  }
  __syncthreads();
  const ModeLayout L{n1};
  const SweepRec helm(rec + L.helm(), n1, lam);
  const SweepRec pois(rec + L.pois(), n1, k2);
  const bool vrow = row < 2;
  const int pv = row & 1;  // v parity (rows 0, 1), u_perp / w parity (rows 2, 3)
  const int po = 1 - pv;
  if (mean) {
    wsweep_T<E>(helm, hw, N, pv, vrow ? Upb : Ub, vrow ? Rb : Rb2, vrow ? W : W2, l);
    if (vrow)
      SP_ROW_PAR(pv, Fpb[n] = -Rb[n];)
    else
      SP_ROW_PAR(pv, Fpp[n] = -Rb2[n];)
  } else {
    // u_par = i D v / k (transposed): A = conj(i) u_par_bar / k on parity po
    if (vrow) SP_ROW_PAR(po, A[n] = mul_i(-Upb[n]) * ik;)
    __syncthreads();
    wderiv_T<E>(N, po, vrow ? A : Ub, vrow ? Tm : Dm, vrow ? W : W2, l);
    __syncthreads();
    if (vrow) SP_ROW_PAR(pv, Vb[n] = Vb[n] + Tm[n];)
    __syncthreads();
    // v = v_p + c_delta v_delta + c_b v_b, (c_delta, c_b) = -Minv (l_a, l_b)
    const double* vdel = rec + L.vdel();
    const double* vbs = rec + L.vb();
    cd ca(0.0), cbb(0.0);
    SP_ROW_PAR(pv, ca = ca + Vb[n] * vdel[n]; cbb = cbb + Vb[n] * vbs[n];)
    ca = row_sum(ca);
    cbb = row_sum(cbb);
    const double* Mi = rec + L.minv() + 4 * pv;
    const cd la = -(ca * Mi[0] + cbb * Mi[2]);
    const cd lb = -(ca * Mi[1] + cbb * Mi[3]);
    const int m = (N % 2 == pv) ? N : N - 1;
    __syncthreads();
    if (vrow) {
      SP_ROW_PAR(pv, Vb[n] = Vb[n] + la * ((double)n * n) + ((n == m) ? lb * lam : cd(0.0));)
      SP_ROW_PAR(po, if (n == N && m == N - 1) Pb[n] = Pb[n] + lb * (2.0 * N);)
    }
    __syncthreads();
    // v_p = H(D P - F_v) on rows 0, 1; u_perp = H(-F_perp) on rows 2, 3
    wsweep_T<E>(helm, hw, N, pv, vrow ? Vb : Ub, vrow ? Rb : Rb2, vrow ? W : W2, l);
    if (vrow)
      SP_ROW_PAR(pv, Fvb[n] = -Rb[n];)
    else
      SP_ROW_PAR(pv, Fpp[n] = -Rb2[n];)
    __syncthreads();
    wderiv_T<E>(N, pv, vrow ? Rb : Ub, vrow ? Tm : Dm, vrow ? W : W2, l);
    __syncthreads();
    if (vrow) SP_ROW_PAR(po, Pb[n] = Pb[n] + Tm[n];)
    __syncthreads();
    // P = Pois(div F), div F = i k F_par + D F_v
    // the rows' operator chosen field by field (a per-lane choice between two
    // records would be made through scratch memory)
    const SweepRec pois_or_helm(rec + (vrow ? L.pois() : L.helm()), n1, vrow ? k2 : lam);
    wsweep_T<E>(pois_or_helm, hw, N, vrow ? po : pv, vrow ? Pb : Ub, vrow ? Db : Dm,
                vrow ? W : W2, l);
    if (vrow) SP_ROW_PAR(po, Fpb[n] = mul_i(-Db[n]) * k;)
    __syncthreads();
    wderiv_T<E>(N, po, vrow ? Db : Ub, vrow ? Tm : Dm, vrow ? W : W2, l);
    __syncthreads();
    if (vrow) SP_ROW_PAR(pv, Fvb[n] = Fvb[n] + Tm[n];)
  }
  __syncthreads();
  // n1 <= 32 E coefficients: a fixed, unrolled pass count
#pragma unroll
  for (int q = 0; q < (32 * E + 63) / 64; ++q) {
    const int n = tid + 64 * q;
    if (n >= n1) break;
    cd gu, gv, gw;
    if (n <= N - 2) {
      if (mean) {
        gu = Fpb[n] * re;
        gw = Fpp[n] * re;
      } else {
        gu = (Fpb[n] * kx + Fpp[n] * kz) * (re * ik);
        gw = (Fpb[n] * kz - Fpp[n] * kx) * (re * ik);
        gv = Fvb[n] * re;
      }
    }
    out[mo + n] = make_double2(gu.re, gu.im);
    out[cs + mo + n] = make_double2(gv.re, gv.im);
    out[2 * cs + mo + n] = make_double2(gw.re, gw.im);
  }
}

// ---------------------------------------------------------------------------
// adj_z: per (y, x) z-line, in place on xp. Reads the three adjoint product
// fields lam (z spectral), forms them in physical space (Hermitian-extended
// inverse FFT of the pair (lam_x + i lam_y) and of lam_z), applies the
// transposed linearised product with the cached base state,
//   du_bar = Omega x lam,  domega_bar = lam x U,
// and returns the six fields to z spectral space (forward FFT of three packed
// pairs, unpacked), scaled by `scale`.
// ---------------------------------------------------------------------------
template <typename R, int PT>
__global__ void __launch_bounds__(256)
    k_adj_z(typename V2<R>::T* __restrict__ xp, const R* __restrict__ base,
            const typename V2<R>::T* __restrict__ tw, FFTPlan1D pl, int ny, int px, int nzm,
            int xc, R scale) {
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
  #pragma unroll 8
  for (int t = threadIdx.x; t < nxl * 2 * pz; t += blockDim.x) {
    const int m = t % pz;
    const int lj = t / pz;  // x_l * 2 + j
    const int jj = lj % 2;
    const int xl = lj / 2;
    const size_t off = ((size_t)y * px + (x0 + xl)) * nzm;
    C val = mk((R)0, (R)0);
    const int fa = (jj == 0) ? 0 : 2;
    if (m < nzm) {
      C a = xp[fa * fs + off + m];
      C b = (jj == 0) ? xp[1 * fs + off + m] : mk((R)0, (R)0);
      if (m == 0) {
        a.y = 0;
        b.y = 0;
      }
      val = mk(a.x - b.y, a.y + b.x);
    } else if (m > pz - nzm) {
      const int mm = pz - m;
      C a = conjc(xp[fa * fs + off + mm]);
      C b = (jj == 0) ? conjc(xp[1 * fs + off + mm]) : mk((R)0, (R)0);
      val = mk(a.x - b.y, a.y + b.x);
    }
    A[lidx<PT>(xl * 3 + jj, m, pz)] = val;
  }
  __syncthreads();
  // inverse FFT of the two used lines of every x (line 2 of each x is idle)
  #pragma unroll 8
  for (int t = threadIdx.x; t < nxl * pz; t += blockDim.x) {
    const int xl = t / pz;
    const int z = t - xl * pz;
    A[lidx<PT>(xl * 3 + 2, z, pz)] = mk((R)0, (R)0);
  }
  __syncthreads();
  C* res = fft_lines<R, PT>(A, B, nxl * 3, pl, twl, (R)1);
  C* oth = (res == A) ? B : A;
  const size_t bs = (size_t)ny * px * pz;
  #pragma unroll 8
  for (int t = threadIdx.x; t < nxl * pz; t += blockDim.x) {
    const int xl = t / pz;
    const int z = t - xl * pz;
    const C p0 = res[lidx<PT>(xl * 3 + 0, z, pz)];
    const C p1 = res[lidx<PT>(xl * 3 + 1, z, pz)];
    const R lx = p0.x, ly = p0.y, lz = p1.x;
    const size_t bo = ((size_t)y * px + (x0 + xl)) * pz + z;
    const R U = base[0 * bs + bo], V = base[1 * bs + bo], W = base[2 * bs + bo];
    const R OX = base[3 * bs + bo], OY = base[4 * bs + bo], OZ = base[5 * bs + bo];
    const R dux = OY * lz - OZ * ly;
    const R duy = OZ * lx - OX * lz;
    const R duz = OX * ly - OY * lx;
    const R dox = ly * W - lz * V;
    const R doy = lz * U - lx * W;
    const R doz = lx * V - ly * U;
    oth[lidx<PT>(xl * 3 + 0, z, pz)] = mk(dux, duy);
    oth[lidx<PT>(xl * 3 + 1, z, pz)] = mk(duz, dox);
    oth[lidx<PT>(xl * 3 + 2, z, pz)] = mk(doy, doz);
  }
  __syncthreads();
  C* fin = fft_lines<R, PT>(oth, res, nxl * 3, pl, twl, (R)-1);
  #pragma unroll 8
  for (int t = threadIdx.x; t < nxl * 3 * nzm; t += blockDim.x) {
    const int m = t % nzm;
    const int lj = t / nzm;
    const int jj = lj % 3;
    const int xl = lj / 3;
    const C a = fin[lidx<PT>(xl * 3 + jj, m, pz)];
    const C am = conjc(fin[lidx<PT>(xl * 3 + jj, (pz - m) % pz, pz)]);
    const C s1 = cscale(cadd(a, am), (R)0.5 * scale);
    const C d = csub(a, am);
    const C s2 = mk(d.y * (R)0.5 * scale, -d.x * (R)0.5 * scale);
    const size_t off = ((size_t)y * px + (x0 + xl)) * nzm + m;
    xp[(2 * jj) * fs + off] = s1;
    xp[(2 * jj + 1) * fs + off] = s2;
  }
}

// ----------------------------------- launchers -----------------------------------


hipError_t launch_stokes_solve_adj(sp_plan* p, const double2* w, double2* out) {
  const Dims& d = p->d;
  const size_t sh = (size_t)p->mode_stride * sizeof(double) + 3 * (size_t)d.ny * sizeof(double) +
                    15 * (size_t)d.ny * sizeof(cd);
  SP_PROF_BEGIN(p, KID_SOLVE_ADJ);
#define SP_SOLVE_ADJ_LAUNCH(EV)                                                                \
  hipLaunchKernelGGL((k_stokes_solve_adj<EV>), dim3(d.nx * d.nzh), dim3(64), sh, p->stream, w, \
                     out, p->d_mode, p->d_hw, p->mode_stride, d.nx, d.ny, d.nzh, d.alpha,       \
                     d.gamma, d.re, d.inv_dt)
  switch (solve_lanes_per_chain(d.ny)) {
    case 1: SP_SOLVE_ADJ_LAUNCH(1); break;
    case 2: SP_SOLVE_ADJ_LAUNCH(2); break;
    case 3: SP_SOLVE_ADJ_LAUNCH(3); break;
    case 4: SP_SOLVE_ADJ_LAUNCH(4); break;
    default: SP_SOLVE_ADJ_LAUNCH(5); break;
  }
#undef SP_SOLVE_ADJ_LAUNCH
  SP_PROF_END(p, KID_SOLVE_ADJ);
  return hipGetLastError();
}

// LDS Stockham fallback for z lengths without a register kernel (zline.hip)
hipError_t launch_adj_z_lds(sp_plan* p, bool fp32) {
  const Dims& d = p->d;
  const size_t el = fp32 ? sizeof(float2) : sizeof(double2);
  const int LL = fft_length_specialised(d.pz) ? line_stride(d.pz) : d.pz;
  int xc = (int)((48 * 1024 - d.pz * el) / (2 * 3 * LL * el));
  if (xc < 1) xc = 1;
  if (xc > d.px) xc = d.px;
  dim3 grid(d.ny, (d.px + xc - 1) / xc);
  const size_t sh = (2 * (size_t)xc * 3 * LL + d.pz) * el;
  const double scale = 1.0 / ((double)d.px * d.pz);
  SP_PROF_BEGIN(p, KID_ADJ_Z);
#define L32(PV)                                                                                   \
  hipLaunchKernelGGL((k_adj_z<float, PV>), grid, dim3(256), sh, p->stream, (float2*)p->xp,        \
                     p->base32, p->f_twz, p->fz, d.ny, d.px, d.nzm, xc, (float)scale)
#define L64(PV)                                                                                   \
  hipLaunchKernelGGL((k_adj_z<double, PV>), grid, dim3(256), sh, p->stream, (double2*)p->xp,      \
                     p->base, p->d_twz, p->fz, d.ny, d.px, d.nzm, xc, scale)
  switch (d.pz) {
    case 12: if (fp32) L32(12); else L64(12); break;
    case 24: if (fp32) L32(24); else L64(24); break;
    case 36: if (fp32) L32(36); else L64(36); break;
    case 48: if (fp32) L32(48); else L64(48); break;
    case 72: if (fp32) L32(72); else L64(72); break;
    case 96: if (fp32) L32(96); else L64(96); break;
    case 144: if (fp32) L32(144); else L64(144); break;
    case 192: if (fp32) L32(192); else L64(192); break;
    default: if (fp32) L32(0); else L64(0); break;
  }
#undef L32
#undef L64
  SP_PROF_END(p, KID_ADJ_Z);
  return hipGetLastError();
}


#define SP_TRY_HIP(expr, what)                 \
  do {                                         \
    sp_status _s = hip_check(p, (expr), what); \
    if (_s != SP_OK) return _s;                \
  } while (0)

sp_status vjp_lin(sp_plan* p, int op, const double2* w, double2* out) {
  if (!p->base_valid) return set_error(p, SP_ERR_INVALID, "no base state: call sp_linearize");
  if (op == SP_OP_RESIDUAL && p->nsteps > 1)
    return set_error(p, SP_ERR_INVALID, "the VJP of the multi-step operator is not provided");
  if (p->advect)
    return set_error(p, SP_ERR_INVALID, "the VJP of the advected step is not provided");
  {
    sp_status s = base_at(p, 0);
    if (s) return s;
  }
  const bool fp32 = (p->precision == SP_MIXED);
  const Dims& d = p->d;
  // the adjoint solve weighs the (0,0) mode of w twice (packed-Euclidean ->
  // Parseval); the transposed synthesis halves it back as it finishes each
  // entry, and forms the residual's (. - w)/dt
  SP_TRY_HIP(launch_stokes_solve_adj(p, w, p->t2), "stokes_solve_adj");
  SP_TRY_HIP(launch_synth_tab(p, p->t2, 1, p->nv, fp32), "analysis^T");
  if (!zline_fuses_x_inverse(p, fp32, 3))
    SP_TRY_HIP(launch_fft_x_inv_gen(p, p->nv, p->xp, 3, 1, fp32), "pad+ifft_x");
  SP_TRY_HIP(launch_adj_z(p, fp32), "adj_z");
  SP_TRY_HIP(launch_fft_x_fwd_gen(p, p->xp, p->yv, 6, fp32), "fft_x+truncate");
  const bool res = (op == SP_OP_RESIDUAL);
  SP_TRY_HIP(launch_adj_synth(p, p->t2, d.inv_dt, res ? d.inv_dt : 1.0, res ? -d.inv_dt : 0.0,
                              res ? w : nullptr, out, fp32),
             "adj_synth");
  return SP_OK;
}

}  // namespace sp

using namespace sp;

extern "C" sp_status sp_vjp_lin(sp_plan* p, int32_t op, const double* w, double* out) {
  if (!p) return SP_ERR_INVALID;
  if (!w || !out) return set_error(p, SP_ERR_INVALID, "null pointer");
  if (op != SP_OP_PHI && op != SP_OP_RESIDUAL) return set_error(p, SP_ERR_INVALID, "bad op");
  if (w == out) return set_error(p, SP_ERR_INVALID, "sp_vjp: out aliases w");
  return vjp_lin(p, op, (const double2*)w, (double2*)out);
}

extern "C" sp_status sp_vjp(sp_plan* p, int32_t op, const double* u, const double* w, double* out) {
  if (!p) return SP_ERR_INVALID;
  if (!u) return set_error(p, SP_ERR_INVALID, "null pointer");
  sp_status s = sp_linearize(p, u);
  if (s) return s;
  return sp_vjp_lin(p, op, w, out);
}
